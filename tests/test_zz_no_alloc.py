"""The allocation-free phi_action against phi_action with a caller workspace.

phi_action_noalloc runs the same kernels as phi_action on the library's own
scratch array (one per GPU, kept between calls).  Two calls in a row, the
second on a smaller operator than the first, must give what phi_action gives
on the same inputs: the same kernels in the same order, so the results are
expected to be bitwise equal; the bar written here is the FP64 parity
tolerance (1e-10 relative) against both phi_action and the oracle.
"""
import numpy as np
import pytest

import synth
from oracle import integrators as I
from oracle import operators as O

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def E(device):
    import paper_1309_4616_amd as E
    E.lib()
    E.noalloc_init(device)
    return E


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _case(E, shape, bc, seed, tau_scale):
    import torch
    h = tuple(1.0 / (n + 1) for n in shape)
    op = E.StencilOp(shape, h, bc)
    A = O.stencil_matrix(shape, h, bc)
    a, b = O.gershgorin_interval(A)
    tau = tau_scale / (b - a)
    v = synth.uniform_vector(A.shape[0], seed)
    vt = torch.as_tensor(v, device="cuda:0")
    return op, A, (a, b), tau, v, vt


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_matches_workspace_call_twice_second_smaller(E, dtype):
    import torch
    # first a 3D grid that runs pair sweeps, then a smaller 2D grid with a
    # ragged row length; the scratch array keeps the first call's contents
    cases = [((40, 36, 30), "neumann0", 3, 13.0), ((37, 29), "dirichlet0", 4, 30.0)]
    sizes = []
    for shape, bc, seed, tau_scale in cases:
        op, A, iv, tau, v, vt = _case(E, shape, bc, seed, tau_scale)
        sizes.append(A.shape[0])
        print(f"noalloc {dtype} {shape} {bc}", flush=True)
        y_na = torch.full_like(vt, float("nan"))
        st_na = E.phi_action_noalloc(op, 1, tau, vt, y_na, tol=TOL, dtype=dtype)
        y_ws, st_ws = E.phi_action(op, 1, tau, vt, tol=TOL, dtype=dtype)
        torch.cuda.synchronize()
        a_na, a_ws = y_na.cpu().numpy(), y_ws.cpu().numpy()
        assert st_na["converged"] == 1
        assert st_na["newton_steps"] == st_ws["newton_steps"]
        assert np.all(np.isfinite(a_na))
        assert relerr(a_na, a_ws) <= TOL
        assert np.array_equal(a_na, a_ws)
        yo, _ = I.phi_action(A, 1, tau, v, TOL, interval=iv)
        assert relerr(a_na, yo) <= (TOL if dtype == "f64" else 5e-6)
    assert sizes[1] < sizes[0]


def test_noalloc_rejects_operator_beyond_scratch(E):
    import torch
    n = 256
    op = E.StencilOp((n, n, n), (1.0 / n,) * 3, "neumann0")
    assert op.workspace_bytes("f64") > E.NOALLOC_SCRATCH_BYTES
    v = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    with pytest.raises(E.ExpiError) as e:
        E.phi_action_noalloc(op, 1, 1e-5, v, v.clone(), tol=TOL)
    assert e.value.name == "EWORKSPACE"
