"""cr_recover_noalloc (the recovery that allocates no device memory) against
cr_recover, through the C ABI (GPU only).

U and P come from the same per-element recovery and must agree bit for bit;
the copy mismatch is the same sum of squares taken in another order (element
order instead of face order), so it agrees to rounding: relative 1e-12.
Two calls in a row, the second on a smaller mesh, check that the partials the
first call left in the static array do not leak into the second.
"""
import numpy as np
import pytest
import torch

import synth
import synth.workloads as wl

pytestmark = pytest.mark.gpu


def _solved(crh, coords, elems, mu, fbar, problem="stokes", method="pcg", ulin=None):
    s = crh.System(coords, elems, mu, 1.0 if problem == "stokes" else 0.01, problem=problem)
    s.eliminate(torch.from_numpy(np.ascontiguousarray(fbar)).cuda(), None,
                None if ulin is None else torch.from_numpy(ulin).cuda())
    s.solve(method, "fp64", tol=1e-11, maxit=200000)
    return s


def _compare(s):
    U0, P0, J0 = s.recover(jump=True)
    U1 = torch.full_like(U0, float("nan"))
    P1 = torch.full_like(P0, float("nan"))
    J1 = torch.full_like(J0, float("nan"))
    before = s._alloc.bytes_in_use
    s.recover_noalloc(U1, P1, J1)
    torch.cuda.synchronize()
    assert s._alloc.bytes_in_use == before  # nothing came from the system's allocator
    assert torch.equal(U0, U1)
    assert torch.equal(P0, P1)
    j0, j1 = J0.item(), J1.item()
    assert np.isfinite(j1) and j1 > 0.0
    assert abs(j1 - j0) <= 1e-12 * j0, (j0, j1)
    # without the mismatch output: same U and P, no scratch used
    U2 = torch.full_like(U0, float("nan"))
    P2 = torch.full_like(P0, float("nan"))
    s.recover_noalloc(U2, P2, None)
    torch.cuda.synchronize()
    assert torch.equal(U0, U2) and torch.equal(P0, P2)
    return j0


def test_noalloc_recover_matches_recover_two_calls_shrinking(gpu):
    # first a 96x96x2 jittered mesh (144 workgroups of partials), then 20x20x2 (7)
    big = wl.square(96, mu=500.0, nu=1.0, jitter=0.2, seed=3, quad=2)
    s = _solved(gpu, big["coords"], big["elems"], big["mu"], big["fbar"])
    _compare(s)
    s.close()
    small = wl.square(20, mu=100.0, nu=1.0, seed=4, quad=2)
    s = _solved(gpu, small["coords"], small["elems"], small["mu"], small["fbar"])
    _compare(s)
    s.close()


def test_noalloc_recover_3d_and_navier_stokes(gpu):
    w = wl.cube(6, mu=100.0)
    s = _solved(gpu, w["coords"], w["elems"], w["mu"], w["fbar"])
    _compare(s)
    s.close()
    w = wl.ns_square(12)
    s = _solved(gpu, w["coords"], w["elems"], 0.0, w["fbar"], problem="ns", method="bicgstab2", ulin=w["ulin"])
    _compare(s)
    s.close()


def test_noalloc_recover_rejects_meshes_above_its_limit(gpu):
    # 1449 x 1449 x 2 = 4,199,202 elements > 4,194,304 = 32768 partials x 128
    coords, elems = synth.square_mesh(1449)
    s = gpu.System(coords, elems, 100.0, 1.0)
    s.eliminate(torch.zeros((len(elems), 2), dtype=torch.float64, device="cuda"))
    U = torch.empty((s.n_int_faces, 2), dtype=torch.float64, device="cuda")
    P = torch.empty((len(elems),), dtype=torch.float64, device="cuda")
    J = torch.empty((1,), dtype=torch.float64, device="cuda")
    with pytest.raises(gpu.CRError, match="limit of 4194304"):
        s.recover_noalloc(U, P, J)
    s.recover_noalloc(U, P, None)  # without the mismatch there is no limit
    torch.cuda.synchronize()
    assert torch.isfinite(P).all()
    s.close()
