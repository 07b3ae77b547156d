// Host-side Leja points and divided differences (plain C++, no HIP).
#pragma once

#include <cfloat>

namespace expi {

constexpr int kMaxLeja = 256;

// Pointer to a table whose first `count` (<= kMaxLeja) entries are the first
// Leja points of [-2, 2]; computed on first need, thread-safe.
const double* leja_points(int count);

// f[xi_0..xi_j], j < count <= kMaxLeja, of f(x) = phi_k(delta (c + gamma x)).
void divided_differences(int k, double delta, double c, double gamma, int count, double* out);

// f[xi_0..xi_j] of f(x) = phi_k(-i delta (c + gamma x)) (complex; real and
// imaginary parts into re, im): the coefficients for phi_k(-i delta H) of a
// Hermitian H with spectrum in [c - 2 gamma, c + 2 gamma].
void divided_differences_skew(int k, double delta, double c, double gamma, int count, double* re,
                              double* im);

// phi_k(z) rounded to double.
double phi_scalar(int k, double z);

}  // namespace expi
