"""GPU parity of the wide-band kernels (factor columns of W = 192 .. 384,
the subdomain sizes of Section 4's own experiments, 300-cell cores) against
the CPU oracle.

Every expected value comes from the oracle: its band LU, local solves,
preconditioner, GMRES and fixed-point iteration; a single subdomain (P = 1,
B^{-1} = A^{-1}) is checked against a sparse direct solve of the oracle's
assembled operator.  Tolerances as for the narrower bands: complex128
within 1e-12, complex64 factors within 2e-5 and applies within 1e-4.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2602_00735_amd as rp
from paper_2602_00735_amd import inputs
from oracle import fem, gmres, ras, richardson
from oracle.geometry import BC_DRCH, Problem

WIDE = {
    # four subdomains of 137 x 137 unknowns: W = 192 (three 64-slot registers)
    "wide": Problem(k=30.0, n_int=230, G=6, Px=2, Py=2, delta=8, kappa=8, sigma=300.0),
    # eight subdomains with W = 118 (register-ring kernels) beside the middle
    # one with W = 192 (wide kernels), in one handle
    "mixed_wide": Problem(k=60.0, n_int=288, G=6, Px=3, Py=3, delta=8, kappa=8, sigma=600.0),
    # RAS-PML-Drch: Dirichlet instead of impedance on the subdomain boundaries
    "wide_drch": Problem(k=30.0, n_int=230, G=6, Px=2, Py=2, delta=8, kappa=8, sigma=300.0,
                         bc=BC_DRCH),
}
_oracles = {}


def oracle_for(name):
    if name not in _oracles:
        _oracles[name] = ras.RasPml(WIDE[name])
    return _oracles[name]


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


@pytest.mark.parametrize("name,precision", [("wide", rp.RAS_MIXED), ("wide", rp.RAS_FP64),
                                            ("mixed_wide", rp.RAS_MIXED)])
def test_wide_factors(name, precision):
    """Column and row copies of L and D^{-1} of every wide subdomain against
    the oracle's band LU (U = D L^T); every slot past the band holds 0."""
    pb = WIDE[name]
    R = oracle_for(name)
    H = setup_gpu(pb, precision)
    tol = 1e-12 if precision == rp.RAS_FP64 else 2e-5
    desc = H.desc()
    wide = [m for m in range(len(desc)) if desc[m][2] > 128]
    assert wide
    for m in wide:
        sd = R.sds[m]
        b, n, W = sd.band, sd.n, desc[m][2]
        assert W % 64 == 0 and W - 64 < b + 1 <= W, (m, W, b)
        npad = (n + 63) // 64 * 64
        Lcols, Lrows, Dinv = rp.ras_pml_export_factor(H, m, npad, W)
        LU = R.batch.factors(m)
        c = np.arange(npad)
        # slots at distance b + 1 .. W from the column (past the band, and
        # the column's own slot) hold zeros
        for dist in range(b + 1, W + 1):
            assert np.all(Lcols[c, (c + dist) % W] == 0), dist
        cc = np.repeat(c, W - 1)
        rr = cc + np.tile(np.arange(1, W), npad)
        ok = rr < npad
        assert np.array_equal(Lrows[rr[ok], cc[ok] % W], Lcols[cc[ok], rr[ok] % W])
        assert np.all(Lrows[c, c % W] == 0)
        D = LU[:, b]
        assert np.abs(1.0 / Dinv[:n] - D).max() <= tol * np.abs(D).max()
        assert np.allclose(Dinv[n:], 1.0)
        for col in range(0, n, max(1, n // 97)):
            for r in range(col + 1, min(col + b + 1, n)):
                ref = LU[r, b + col - r]
                assert abs(Lcols[col, r % W] - ref) <= tol * max(1.0, abs(ref)), (m, r, col)


@pytest.mark.parametrize("name", list(WIDE))
@pytest.mark.parametrize("precision,tol", [(rp.RAS_FP64, 1e-12), (rp.RAS_MIXED, 1e-4)])
def test_wide_local_solves_and_apply(name, precision, tol):
    pb = WIDE[name]
    R = oracle_for(name)
    H = setup_gpu(pb, precision)
    v = inputs.random_vector(pb.ndof, 11)
    xl = torch.zeros(H.nloc, dtype=torch.complex128, device="cuda")
    rp.ras_pml_local_solve(H, dev(v), xl)
    got = host(xl)
    ref = R.local_solve(v)
    # complex64 factors: a single local solve carries the local operator's
    # condition number (3e-4 on the 116-cell corner subdomains at k = 30,
    # h = 1/288); the preconditioner's sum below is held to 1e-4
    ltol = tol if precision == rp.RAS_FP64 else 1e-3
    for m in range(len(R.sds)):
        err = relerr(R.local_part(got, m), R.local_part(ref, m))
        assert err <= ltol, (name, m, err)
    for seed in (1, 2):
        v = inputs.random_vector(pb.ndof, seed)
        z = torch.zeros(pb.ndof, dtype=torch.complex128, device="cuda")
        rp.ras_pml_apply(H, dev(v), z)
        err = relerr(host(z), R.apply(v))
        assert err <= tol, (name, precision, err)


@pytest.mark.parametrize("name", list(WIDE))
@pytest.mark.parametrize("precision", [rp.RAS_FP64, rp.RAS_MIXED])
def test_wide_gmres_matches_oracle(name, precision):
    pb = WIDE[name]
    R = oracle_for(name)
    b = fem.rhs(R.M1, inputs.centre_gaussian(pb.n_int, pb.G, 0.1))
    ref = gmres.gmres(lambda x: R.A @ x, R.apply, b, rtol=1e-6, restart=100, maxit=500)
    tight = gmres.gmres(lambda x: R.A @ x, R.apply, b, rtol=1e-12, restart=100, maxit=500)
    assert tight.converged
    H = setup_gpu(pb, precision)
    x = torch.zeros(pb.ndof, dtype=torch.complex128, device="cuda")
    rc, it, rr, hist = rp.gmres_solve(H, dev(b), x, rtol=1e-6, restart=100, maxit=500)
    assert rc == rp.RAS_OK
    xs = host(x)
    assert np.linalg.norm(b - R.A @ xs) <= 1e-6 * np.linalg.norm(b) * (1 + 1e-9)
    if precision == rp.RAS_FP64:
        assert abs(it - ref.iters) <= 1, (it, ref.iters)
        if it == ref.iters:
            assert relerr(xs, ref.x) <= 1e-10
        k = min(len(ref.history), len(hist) - 1)
        assert np.allclose(hist[1:k + 1], ref.history[:k], rtol=1e-6, atol=1e-14)
    else:
        # complex64 factors cost iterations on this finer mesh (k h = 0.13):
        # the oracle's GMRES with its factors rounded to complex64 (a
        # one-column LDL^T in complex64 arithmetic) takes 21 steps on "wide"
        # against 14 in complex128
        assert ref.iters - 2 <= it <= ref.iters + 8, (it, ref.iters)
    assert relerr(xs, ref.x) <= 1e-5
    assert relerr(xs, tight.x) <= 1e-5


def test_wide_richardson_fp64_matches_oracle():
    """Algorithm 1 with a wide middle subdomain: every iterate's residual."""
    pb = WIDE["mixed_wide"]
    R = oracle_for("mixed_wide")
    b = fem.rhs(R.M1, inputs.centre_gaussian(pb.n_int, pb.G, 0.1))
    ref = richardson.ras_richardson(lambda y: R.A @ y, R.apply, b, rtol=1e-6, maxit=60)
    H = setup_gpu(pb, rp.RAS_FP64)
    x = torch.zeros(pb.ndof, dtype=torch.complex128, device="cuda")
    rc, it, rr, hist = rp.ras_pml_richardson(H, dev(b), x, rtol=1e-6, maxit=60)
    assert rc == (rp.RAS_OK if ref.converged else rp.RAS_ENOTCONV)
    assert it == ref.iters
    assert np.allclose(hist, ref.history, rtol=1e-8, atol=1e-15)
    assert relerr(host(x), ref.x) <= 1e-9


# One subdomain (B^{-1} = A^{-1}): W = 256, 320, 384 and 448 (n_fast 205,
# 265, 351, 431), against a sparse direct solve.  In complex64 the solve of these
# single large operators is backward stable but its forward error carries
# the condition number: a one-column LDL^T in complex64 arithmetic (on the
# CPU) leaves normwise backward errors of 1.6e-7 .. 2.1e-7 and forward
# errors of 5.4e-5, 3.4e-4 and 1.5e-3 (up to n_fast 351; the blocked kernel
# measured 3.7e-2 at n_fast 431); the test bounds the backward error by ten
# times that and checks the forward error only for sanity (1e-1).
@pytest.mark.parametrize("n_int", [194, 254, 340, 420])
@pytest.mark.parametrize("precision", [rp.RAS_FP64, rp.RAS_MIXED])
def test_wide_single_subdomain_is_the_direct_solve(n_int, precision):
    import scipy.sparse.linalg as spla
    pb = Problem(k=40.0, n_int=n_int, G=6, Px=1, Py=1, delta=0, kappa=0, sigma=400.0)
    A, M1 = fem.assemble_global(pb)
    H = setup_gpu(pb, precision)
    assert H.desc()[0][2] == {194: 256, 254: 320, 340: 384, 420: 448}[n_int]
    v = inputs.random_vector(pb.ndof, 3)
    z = torch.zeros(pb.ndof, dtype=torch.complex128, device="cuda")
    rp.ras_pml_apply(H, dev(v), z)
    ref = spla.spsolve(A.tocsc(), v)
    zs = host(z)
    if precision == rp.RAS_FP64:
        assert relerr(zs, ref) <= 1e-10
    else:
        a_inf = abs(A).sum(axis=1).max()
        back = np.linalg.norm(A @ zs - v) / (a_inf * np.linalg.norm(zs))
        assert back <= 2e-6, back
        assert relerr(zs, ref) <= 1e-1
    # GMRES with the exact inverse as preconditioner: one iteration (FP64)
    b = fem.rhs(M1, inputs.centre_gaussian(pb.n_int, pb.G, 0.1))
    x = torch.zeros(pb.ndof, dtype=torch.complex128, device="cuda")
    rc, it, rr, _ = rp.gmres_solve(H, dev(b), x, rtol=1e-8, restart=20, maxit=50)
    assert rc == rp.RAS_OK
    if precision == rp.RAS_FP64:
        assert it == 1 and rr <= 1e-10
    else:
        assert it <= 4


@pytest.mark.parametrize("solver,precision", [("richardson", rp.RAS_MIXED),
                                              ("gmres", rp.RAS_MIXED),
                                              ("richardson", rp.RAS_FP64)])
def test_table4_covering_at_k300(solver, precision):
    """Section 4's own covering at k = 300: grid 600^2, 2 x 2 subdomains with
    300-cell cores, overlap 4 and PML 12 cells (the width rule), a global PML
    of three wavelengths, the smoothed point source, rtol 1e-10 (Table 4
    reports 7 Richardson steps).  Through the wide kernels (W = 384), in
    mixed precision and in FP64, checked by the true residual under the
    oracle's assembled operator (its band LU of four 124k-unknown subdomains
    would take minutes)."""
    pb = Problem(k=300.0, n_int=600, G=37, Px=2, Py=2, delta=4, kappa=12, sigma=3000.0)
    A, M1 = fem.assemble_global(pb)
    b = fem.rhs(M1, inputs.paper(pb.k, pb.n_int, pb.G))
    H = setup_gpu(pb, precision)
    assert all(d[2] == 384 for d in H.desc())
    x = torch.zeros(pb.ndof, dtype=torch.complex128, device="cuda")
    if solver == "richardson":
        rc, it, rr, _ = rp.ras_pml_richardson(H, dev(b), x, rtol=1e-10, maxit=50)
    else:
        rc, it, rr, _ = rp.gmres_solve(H, dev(b), x, rtol=1e-10, restart=100, maxit=50)
    assert rc == rp.RAS_OK and it <= 10, (rc, it)
    xs = host(x)
    assert np.linalg.norm(b - A @ xs) <= 1e-10 * np.linalg.norm(b) * (1 + 1e-6)


def test_wide_and_narrow_problems_in_one_batch():
    """A batch handle holding a problem of wide subdomains (W = 192) and one
    of narrow ones (register-ring kernels): the fixed-point iteration of each
    equals its own oracle run (FP64), step for step."""
    pbs = [Problem(k=30.0, n_int=230, G=8, Px=2, Py=2, delta=8, kappa=8, sigma=300.0),
           Problem(k=20.0, n_int=40, G=6, Px=2, Py=2, delta=6, kappa=6, sigma=200.0)]
    o = rp.default_opts(precision=rp.RAS_FP64)
    H = rp.ras_pml_setup_batch([p.k for p in pbs], [1 / p.n_int for p in pbs],
                               [(p.n_int, p.n_int) for p in pbs], [(p.Px, p.Py) for p in pbs],
                               [p.delta for p in pbs], [p.kappa for p in pbs], o)
    assert sorted({d[2] > 128 for d in H.desc()}) == [False, True]
    Rs = [ras.RasPml(p) for p in pbs]
    bs = [fem.rhs(R.M1, inputs.centre_gaussian(p.n_int, p.G, 0.1)) for p, R in zip(pbs, Rs)]
    refs = [richardson.ras_richardson(lambda y, R=R: R.A @ y, R.apply, b, rtol=1e-6, maxit=80)
            for R, b in zip(Rs, bs)]
    x = torch.zeros(H.ndof, dtype=torch.complex128, device="cuda")
    rc, it, rr, hist = rp.ras_pml_richardson(H, dev(np.concatenate(bs)), x, rtol=1e-6, maxit=80)
    assert it == max(r.iters for r in refs)
    xs = host(x)
    for p, ref in enumerate(refs):
        off, m = H.problem_offset(p)
        itp, rrp, conv = rp.ras_pml_batch_result(H, p)
        assert itp == ref.iters and conv == ref.converged
        assert abs(rrp - ref.relres) <= 1e-8 * ref.relres
        assert relerr(xs[off:off + m], ref.x) <= 1e-9


def test_wide_graph_replayed_steps_and_autotune():
    """The FGMRES steps replayed from the recorded HIP graph (wide band-solve
    launches included) equal the eager steps bit for bit; the autotuner runs
    on a handle whose subdomains are all wide, and the apply afterwards is
    unchanged (its factorisation has no variants to choose)."""
    pb = WIDE["mixed_wide"]
    R = oracle_for("mixed_wide")
    b = dev(fem.rhs(R.M1, inputs.centre_gaussian(pb.n_int, pb.G, 0.1)))
    res = []
    for flags in (0, rp.RAS_FLAG_GRAPH_STEPS):
        o = rp.default_opts(sigma=pb.sigma, global_pml=pb.G, precision=rp.RAS_MIXED, flags=flags)
        H = rp.ras_pml_setup(pb.k, 1.0 / pb.n_int, (pb.n_int, pb.n_int), (pb.Px, pb.Py),
                             pb.delta, pb.kappa, o)
        x = torch.zeros_like(b)
        rc, it, rr, hist = rp.gmres_solve(H, b, x, rtol=1e-6, restart=16, maxit=500)
        assert rc == rp.RAS_OK
        res.append((it, rr, np.asarray(hist).copy(), host(x)))
        H.close()
    (it0, rr0, h0, x0), (it1, rr1, h1, x1) = res
    assert it0 == it1 and rr0 == rr1 and np.array_equal(h0, h1) and np.array_equal(x0, x1)
    # the autotuner on an all-wide handle
    import os
    import tempfile
    pw = WIDE["wide"]
    H = setup_gpu(pw, rp.RAS_MIXED)
    v = dev(inputs.random_vector(pw.ndof, 5))
    z0 = torch.zeros_like(v)
    rp.ras_pml_apply(H, v, z0)
    path = os.path.join(tempfile.mkdtemp(), "tune.json")
    rp.ras_pml_autotune(H, path)
    z1 = torch.zeros_like(v)
    rp.ras_pml_apply(H, v, z1)
    assert torch.equal(z0, z1)
    assert rp.ras_pml_tuning(H)["ldlt"] == []
