"""ras_pml_richardson_noalloc (every buffer of the fixed-point solve in the
library's static scratch array) against ras_pml_richardson (the handle's own
buffers), through the C ABI.  The two run the same kernels in the same
order, so the iterates, step counts and residual histories must be equal bit
for bit; calls follow each other with smaller inputs (the scratch keeps the
previous call's contents), and sizes beyond the scratch are refused on the
host."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2602_00735_amd as rp
from paper_2602_00735_amd import inputs
from oracle import geometry
from oracle.geometry import Problem


@pytest.fixture(scope="module", autouse=True)
def gpu_available():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rp.lib()


def setup(pbs, precision):
    o = rp.default_opts(precision=precision, global_pml=pbs[0].G, sigma=pbs[0].sigma)
    if len(pbs) == 1:
        p = pbs[0]
        return rp.ras_pml_setup(p.k, 1.0 / p.n_int, (p.n_int, p.n_int), (p.Px, p.Py), p.delta,
                                p.kappa, o)
    return rp.ras_pml_setup_batch([p.k for p in pbs], [1 / p.n_int for p in pbs],
                                  [(p.n_int, p.n_int) for p in pbs], [(p.Px, p.Py) for p in pbs],
                                  [p.delta for p in pbs], [p.kappa for p in pbs],
                                  rp.default_opts(precision=precision))


def rhs(H, pbs):
    """b = M f for a Gaussian of width 0.1 in every problem (device)."""
    f = np.concatenate([inputs.centre_gaussian(p.n_int, p.G, 0.1) for p in pbs])
    fd = torch.from_numpy(f).to("cuda")
    b = torch.zeros_like(fd)
    rp.ras_pml_rhs(H, fd, b)
    return b


def both(H, b, rtol, maxit, x0=None):
    out = []
    for fn in (rp.ras_pml_richardson, rp.ras_pml_richardson_noalloc):
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        rc, it, rr, hist = fn(H, b, x, rtol=rtol, maxit=maxit)
        torch.cuda.synchronize()
        per = [rp.ras_pml_batch_result(H, p) for p in range(H.nprob)]
        out.append((rc, it, rr, hist.copy(), x.cpu().numpy(), per))
    return out


def assert_equal(a, e):
    rc, it, rr, hist, x, per = a
    assert (rc, it, per) == (e[0], e[1], e[5])
    assert rr == e[2]
    assert np.array_equal(hist, e[3])
    assert np.array_equal(x, e[4])


def test_noalloc_equals_handle_buffers_on_shrinking_inputs():
    k160 = geometry.config_problem("k160")
    k20 = geometry.config_problem("k20")
    base = [k20, Problem(k=12.0, n_int=45, G=3, Px=3, Py=4, delta=3, kappa=3, sigma=120.0),
            Problem(k=40.0, n_int=80, G=8, Px=2, Py=2, delta=8, kappa=8, sigma=400.0)]
    batch = [Problem(k=p.k, n_int=p.n_int, G=p.kappa, Px=p.Px, Py=p.Py, delta=p.delta,
                     kappa=p.kappa, sigma=10 * p.k) for p in base]
    # largest first: each later call finds the previous call's data in the
    # scratch (and its counters at other offsets)
    cases = [("k160 mixed", [k160], rp.RAS_MIXED, 1e-6, 200),
             ("k20 fp64", [k20], rp.RAS_FP64, 1e-8, 100),
             ("batch of 3 fp64 (one stagnates)", batch, rp.RAS_FP64, 1e-6, 30),
             ("k20 mixed from a random x0", [k20], rp.RAS_MIXED, 1e-6, 50)]
    sizes = []
    for name, pbs, prec, rtol, maxit in cases:
        print("case:", name, flush=True)
        H = setup(pbs, prec)
        sizes.append(H.ndof)
        b = rhs(H, pbs)
        x0 = None
        if "random" in name:
            x0 = torch.from_numpy(inputs.random_vector(H.ndof, 5)).to("cuda")
        a, e = both(H, b, rtol, maxit, x0)
        assert a[0] in (rp.RAS_OK, rp.RAS_ENOTCONV) and a[1] > 0
        assert_equal(e, a)
        H.close()
    assert sizes[1] < sizes[0]


def test_noalloc_refuses_what_the_scratch_cannot_hold():
    pb = geometry.config_problem("k20")
    H = setup([pb], rp.RAS_FP64)
    b = rhs(H, [pb])
    x = torch.zeros_like(b)
    # the residual history of 10^7 steps (80 MB) exceeds the 64 MiB scratch:
    # refused on the host before any launch, x untouched
    rc, it, rr, hist = rp.ras_pml_richardson_noalloc(H, b, x, rtol=1e-6, maxit=10_000_000,
                                                     check=False)
    assert rc == rp.RAS_EINVAL and it == 0
    assert b"scratch" in rp.lib().ras_pml_last_error(H.ptr)
    assert torch.count_nonzero(x) == 0
    # the same handle then solves normally
    rc, it, *_ = rp.ras_pml_richardson_noalloc(H, b, x, rtol=1e-6, maxit=100)
    assert rc == rp.RAS_OK and it > 0
    H.close()
