// Host-side interpolation data: real Leja points of [-2, 2] and the Newton
// divided differences of the phi functions at them (Sec. III-C: the matrix
// functions are evaluated by interpolation at Leja points; Sec. II-C: the
// interpolant is applied through products (alpha A + beta I) x).
//
// Plain C++ (no HIP), extended precision (x86 long double, 64-bit mantissa).
#include "leja.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <mutex>
#include <vector>

namespace expi {

namespace {

typedef long double ld;

// Local maximiser of sum_j log|x - p_j| strictly inside (lo, hi), where lo
// and hi are consecutive points of the set.  Its derivative
// D(x) = sum_j 1/(x - p_j) falls strictly from +inf to -inf on the gap, so
// the maximiser is the unique root of D; safeguarded Newton (D' < 0) with a
// bisection bracket, started at `start`.
ld gap_maximiser(const std::vector<ld>& pts, ld lo, ld hi, ld start) {
    ld a = lo, b = hi;
    ld x = (start > a && start < b) ? start : 0.5L * (a + b);
    for (int it = 0; it < 200; ++it) {
        ld d = 0.0L, dd = 0.0L;
        for (ld p : pts) {
            ld r = 1.0L / (x - p);
            d += r;
            dd -= r * r;
        }
        if (d > 0) a = x; else b = x;
        ld xn = x - d / dd;
        if (!(xn > a && xn < b)) xn = 0.5L * (a + b);
        if (std::fabs(xn - x) <= 4.0L * LDBL_EPSILON * std::fabs(x) + LDBL_MIN || b - a <= 0) {
            x = xn;
            break;
        }
        x = xn;
    }
    return x;
}

// The table grows on demand (the sequence is prefix-stable, so extending it
// never changes earlier points).  Growth happens under a mutex; readers only
// touch entries below the published count.
struct LejaTable {
    std::mutex mu;
    std::atomic<int> count{0};
    double pts[kMaxLeja];
    std::vector<ld> set, sorted, guess;
};

LejaTable g_table;

void extend_table(int want) {
    LejaTable& t = g_table;
    if (t.set.empty()) {
        t.set = {2.0L, -2.0L};
        t.sorted = {-2.0L, 2.0L};
        t.guess = {0.0L};
    }
    while ((int)t.set.size() < want) {
        std::vector<ld>& pts = t.set;
        ld best_x = 0, best_v = -INFINITY;
        int best_g = -1;
        std::vector<ld> cand(t.sorted.size() - 1);
        std::vector<ld> val(t.sorted.size() - 1);
        for (size_t g = 0; g + 1 < t.sorted.size(); ++g) {
            ld x = gap_maximiser(pts, t.sorted[g], t.sorted[g + 1], t.guess[g]);
            ld v = 0.0L;
            for (ld p : pts) v += std::log(std::fabs(x - p));
            cand[g] = x;
            val[g] = v;
            if (v > best_v) { best_v = v; best_x = x; best_g = (int)g; }
        }
        // ties (within a relative 1e-10 of the log-product) go to the larger point
        for (size_t g = 0; g < cand.size(); ++g) {
            if (std::fabs(val[g] - best_v) <= 1e-10L * std::max(1.0L, std::fabs(best_v)) &&
                cand[g] > best_x) {
                best_x = cand[g];
                best_g = (int)g;
            }
        }
        pts.push_back(best_x);
        // split gap best_g at the new point; every other gap keeps its last
        // maximiser as the start value of the next search
        ld lo = t.sorted[best_g], hi = t.sorted[best_g + 1];
        t.sorted.insert(t.sorted.begin() + best_g + 1, best_x);
        std::vector<ld> next;
        next.reserve(cand.size() + 1);
        for (int g = 0; g < (int)cand.size(); ++g) {
            if (g == best_g) {
                next.push_back(0.5L * (lo + best_x));
                next.push_back(0.5L * (best_x + hi));
            } else {
                next.push_back(cand[g]);
            }
        }
        t.guess.swap(next);
    }
    int have = t.count.load(std::memory_order_relaxed);
    for (int i = have; i < want; ++i) t.pts[i] = (double)t.set[i];
    t.count.store(want, std::memory_order_release);
}

// phi_k(z) in long double: phi_0 = exp; for k >= 1 the power series
// sum_i z^i/(i+k)! when |z| < 1, else phi_1 = expm1(z)/z and
// phi_{j+1} = (phi_j - 1/j!)/z.
ld phi_ld(int k, ld z) {
    if (k == 0) return std::exp(z);
    if (std::fabs(z) < 1.0L) {
        ld fact = 1.0L;
        for (int i = 2; i <= k; ++i) fact *= (ld)i;
        ld term = 1.0L / fact, sum = term;
        for (int i = 1; i < 200; ++i) {
            term *= z / (ld)(i + k);
            sum += term;
            if (std::fabs(term) <= 1e-22L * std::fabs(sum)) break;
        }
        return sum;
    }
    ld val = std::expm1(z) / z;
    ld fact = 1.0L;
    for (int j = 1; j < k; ++j) {
        fact *= (ld)j;  // j!
        val = (val - 1.0L / fact) / z;
    }
    return val;
}

// phi_k(z) for complex z in long double: the power series for |z| < 1,
// else (e^z - 1)/z and the same recurrence (no cancellation there).
typedef std::complex<ld> cld;
cld phi_cld(int k, cld z) {
    if (k == 0) return std::exp(z);
    if (std::abs(z) < 1.0L) {
        ld fact = 1.0L;
        for (int i = 2; i <= k; ++i) fact *= (ld)i;
        cld term = 1.0L / fact, sum = term;
        for (int i = 1; i < 200; ++i) {
            term *= z / (ld)(i + k);
            sum += term;
            if (std::abs(term) <= 1e-22L * std::abs(sum)) break;
        }
        return sum;
    }
    cld val = (std::exp(z) - 1.0L) / z;
    ld fact = 1.0L;
    for (int j = 1; j < k; ++j) {
        fact *= (ld)j;
        val = (val - 1.0L / fact) / z;
    }
    return val;
}

}  // namespace

void divided_differences_skew(int k, double delta, double c, double gamma, int count, double* re,
                              double* im) {
    const double* xi = leja_points(count);
    std::vector<cld> d(count);
    std::vector<ld> x(count);
    for (int i = 0; i < count; ++i) {
        x[i] = (ld)xi[i];
        d[i] = phi_cld(k, cld(0.0L, -(ld)delta * ((ld)c + (ld)gamma * x[i])));
    }
    for (int j = 1; j < count; ++j)
        for (int i = count - 1; i >= j; --i) d[i] = (d[i] - d[i - 1]) / (x[i] - x[i - j]);
    for (int i = 0; i < count; ++i) {
        re[i] = (double)d[i].real();
        im[i] = (double)d[i].imag();
    }
}

const double* leja_points(int count) {
    if (count > kMaxLeja) count = kMaxLeja;
    if (g_table.count.load(std::memory_order_acquire) < count) {
        std::lock_guard<std::mutex> lock(g_table.mu);
        if (g_table.count.load(std::memory_order_acquire) < count)
            extend_table(std::max(count, 2));
    }
    return g_table.pts;
}

void divided_differences(int k, double delta, double c, double gamma, int count, double* out) {
    const double* xi = leja_points(count);
    std::vector<ld> d(count), x(count);
    for (int i = 0; i < count; ++i) {
        x[i] = (ld)xi[i];
        d[i] = phi_ld(k, (ld)delta * ((ld)c + (ld)gamma * x[i]));
    }
    for (int j = 1; j < count; ++j)
        for (int i = count - 1; i >= j; --i) d[i] = (d[i] - d[i - 1]) / (x[i] - x[i - j]);
    for (int i = 0; i < count; ++i) out[i] = (double)d[i];
}

double phi_scalar(int k, double z) { return (double)phi_ld(k, (ld)z); }

}  // namespace expi
