"""GPU solutions at full workload sizes against whole oracle solves.

The benchmark's workload (k = 640, h = 1/1280, 32 x 32 subdomains, the
Gaussian source of width 0.05) is solved by the oracle's own RAS-PML GMRES
(complex128, every subdomain factorised, textbook right-preconditioned
GMRES(100), rtol 1e-6) and by the library in both precisions; the solutions
must agree within 1e-5 relative l2 and the step counts within +-2 (FP64: +-1).
The paper's own source (Section 4: the smoothed point source
(16 k^2/pi^3) exp(-16 k^2 |x - x_c|^2 / pi^2), which radiates at every k) is
solved at k = 160 by GMRES and by the fixed-point iteration of Algorithm 1,
in both precisions, against the oracle's whole solves.

These tests spend most of their time in the CPU oracle (about a minute at
k = 640 on 16 host threads); they hold its factors (26 GB) only while the
module runs.
"""
import gc

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

import paper_2602_00735_amd as rp
from paper_2602_00735_amd import inputs
from oracle import fem, geometry, gmres, ras, richardson


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def setup_gpu(pb, precision):
    o = rp.default_opts(sigma=pb.sigma, global_pml=pb.G, bc=pb.bc, pou=pb.pou,
                        precision=precision)
    return rp.ras_pml_setup(pb.k, 1.0 / pb.n_int, (pb.n_int, pb.n_int), (pb.Px, pb.Py),
                            pb.delta, pb.kappa, o)


@pytest.fixture(scope="module", autouse=True)
def gpu_available():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rp.lib()


def gpu_solve(pb, f, precision, solver="gmres", rtol=1e-6):
    """Right-hand side b = M f on the device and one solve from x0 = 0."""
    H = setup_gpu(pb, precision)
    fd = dev(f)
    b = torch.zeros_like(fd)
    rp.ras_pml_rhs(H, fd, b)
    x = torch.zeros_like(fd)
    if solver == "gmres":
        rc, it, rr, hist = rp.gmres_solve(H, b, x, rtol=rtol, restart=100, maxit=500)
    else:
        rc, it, rr, hist = rp.ras_pml_richardson(H, b, x, rtol=rtol, maxit=500)
    out = dict(rc=rc, iters=it, relres=rr, hist=hist, x=host(x), b=host(b))
    H.close()
    return out


# ------------------------------------------------------------------ k = 640
@pytest.fixture(scope="module")
def k640_oracle():
    pb = geometry.config_problem("k640")
    R = ras.RasPml(pb)
    f = inputs.centre_gaussian(pb.n_int, pb.G, 0.05)
    b = fem.rhs(R.M1, f)
    ref = gmres.gmres(lambda x: R.A @ x, R.apply, b, rtol=1e-6, restart=100, maxit=500)
    assert ref.converged
    yield pb, R.A, f, b, ref
    del R
    gc.collect()


@pytest.mark.parametrize("precision,dit", [(rp.RAS_MIXED, 2), (rp.RAS_FP64, 1)])
def test_k640_gmres_against_the_full_oracle_solve(k640_oracle, precision, dit):
    """The headline workload: the library's solution within 1e-5 relative l2
    of the oracle's GMRES solution at the same tolerance."""
    pb, A, f, b, ref = k640_oracle
    g = gpu_solve(pb, f, precision)
    assert g["rc"] == rp.RAS_OK and g["relres"] <= 1e-6
    assert np.linalg.norm(g["b"] - b) <= 1e-12 * np.linalg.norm(b)
    assert abs(g["iters"] - ref.iters) <= dit, (g["iters"], ref.iters)
    assert np.linalg.norm(b - A @ g["x"]) <= 1e-6 * np.linalg.norm(b) * (1 + 1e-9)
    err = relerr(g["x"], ref.x)
    print("k640 precision=%d iters=%d (oracle %d) error vs oracle %.3e"
          % (precision, g["iters"], ref.iters, err), flush=True)
    assert err <= 1e-5
    if precision == rp.RAS_FP64 and g["iters"] == ref.iters:
        assert err <= 1e-9


# ------------------------------------------------------------------ k = 160, paper source
@pytest.fixture(scope="module")
def k160_paper():
    """k = 160, h = 1/320, 16 x 16 subdomains, the Section 4 source; the
    oracle's GMRES(100) and fixed-point solves to rtol 1e-6."""
    pb = geometry.config_problem("k160")
    R = ras.RasPml(pb)
    f = inputs.paper(pb.k, pb.n_int, pb.G)
    b = fem.rhs(R.M1, f)
    ref_g = gmres.gmres(lambda x: R.A @ x, R.apply, b, rtol=1e-6, restart=100, maxit=500)
    ref_r = richardson.ras_richardson(lambda x: R.A @ x, R.apply, b, rtol=1e-6, maxit=500)
    assert ref_g.converged and ref_r.converged
    yield pb, R.A, f, b, ref_g, ref_r
    del R
    gc.collect()


@pytest.mark.parametrize("precision,dit", [(rp.RAS_MIXED, 2), (rp.RAS_FP64, 1)])
def test_k160_paper_source_gmres_against_the_full_oracle_solve(k160_paper, precision, dit):
    pb, A, f, b, ref, _ = k160_paper
    g = gpu_solve(pb, f, precision)
    assert g["rc"] == rp.RAS_OK
    assert abs(g["iters"] - ref.iters) <= dit, (g["iters"], ref.iters)
    assert np.linalg.norm(b - A @ g["x"]) <= 1e-6 * np.linalg.norm(b) * (1 + 1e-9)
    assert relerr(g["x"], ref.x) <= 1e-5
    if precision == rp.RAS_FP64:
        if g["iters"] == ref.iters:
            assert relerr(g["x"], ref.x) <= 1e-9
        # the residual estimates agree step by step
        k = min(len(ref.history), len(g["hist"]) - 1)
        assert np.allclose(g["hist"][1:k + 1], ref.history[:k], rtol=1e-6, atol=1e-14)


@pytest.mark.parametrize("precision", [rp.RAS_MIXED, rp.RAS_FP64])
def test_k160_paper_source_richardson_against_the_full_oracle_solve(k160_paper, precision):
    """Algorithm 1 on the radiating field: FP64 takes the oracle's step count
    with every iterate's residual within 1e-8; mixed within +-2 steps; both
    solutions within 1e-5 of the oracle's."""
    pb, A, f, b, _, ref = k160_paper
    g = gpu_solve(pb, f, precision, solver="richardson")
    assert g["rc"] == rp.RAS_OK
    if precision == rp.RAS_FP64:
        assert g["iters"] == ref.iters
        assert np.allclose(g["hist"], ref.history, rtol=1e-8, atol=0)
    else:
        assert abs(g["iters"] - ref.iters) <= 2, (g["iters"], ref.iters)
    assert np.linalg.norm(b - A @ g["x"]) <= 1e-6 * np.linalg.norm(b) * (1 + 1e-9)
    assert relerr(g["x"], ref.x) <= 1e-5
