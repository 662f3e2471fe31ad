"""GPU parity of the learned warm start against the float64 oracle.

Tolerances: the network computes in bfloat16 (8-bit significand, unit
roundoff 2^-9 = 2e-3) with fp32 accumulation; the deepest path rounds the
activations about 20 times (forward) and the gradients as often again, so
relative l2 errors of ~1e-2 are expected: 3e-2 for outputs and the loss,
6e-2 for weight gradients.  Adam runs in fp32 (1e-5).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_2602_00735_amd as rp
from paper_2602_00735_amd import inputs
from oracle import fem, geometry, ras
from oracle import warmstart as ows
from oracle.geometry import Problem

CH = (8, 16, 24, 32, 32)        # padded to 16/16/32/32/32: every tile count occurs


@pytest.fixture(scope="module", autouse=True)
def gpu_available():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rp.lib()


def as_dict(flat, channels):
    out, off = {}, 0
    for name, (ci, co) in zip(rp.WS_LAYERS, rp.ws_shapes(channels)):
        n = 9 * ci * co
        out[name] = flat[off:off + n].astype(np.float64).reshape(3, 3, ci, co)
        off += n
    return out


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def setup(grid=32, B=3, seed=0, channels=CH):
    flat = inputs.ws_init_weights(rp.ws_shapes(channels), seed)
    rng = np.random.default_rng(100 + seed)
    x = rng.standard_normal((B, grid, grid, 2)).astype(np.float32)
    t = rng.standard_normal((B, grid, grid, 2)).astype(np.float32)
    net = rp.WSNet(grid, channels, B)
    net.set_weights(flat)
    return net, flat, x, t


def test_weights_round_trip_and_sizes():
    net, flat, _, _ = setup()
    assert net.nweights == sum(9 * ci * co for ci, co in rp.ws_shapes(CH))
    assert np.array_equal(net.get_weights(), flat)
    with pytest.raises(rp.RasPmlError):
        rp.WSNet(40, CH, 2)             # grid not divisible by 16
    with pytest.raises(rp.RasPmlError):
        rp.WSNet(32, (8, 16, 24, 32, 16), 2)   # c3 != c4


@pytest.mark.parametrize("grid,B,seed", [(32, 3, 0), (48, 2, 1)])
def test_forward_matches_oracle(grid, B, seed):
    net, flat, x, _ = setup(grid, B, seed)
    y = net.forward(torch.from_numpy(x).cuda())
    ref, _ = ows.forward(as_dict(flat, CH), x.astype(np.float64))
    got = y.cpu().numpy()
    assert relerr(got, ref) <= 3e-2, relerr(got, ref)
    # each sample on its own gives the same values as in the batch
    y1 = net.forward(torch.from_numpy(x[1:2].copy()).cuda())
    assert torch.equal(y1[0], y[1])


def test_gradient_matches_oracle():
    net, flat, x, t = setup(32, 3, 2)
    loss, g = net.gradient(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    params = as_dict(flat, CH)
    yref, tape = ows.forward(params, x.astype(np.float64))
    lref = ows.loss(yref, t.astype(np.float64))
    gref = ows.backward(params, tape, t.astype(np.float64))
    assert abs(loss - lref) <= 3e-2 * lref
    gd = as_dict(g, CH)
    for name in rp.WS_LAYERS:
        assert relerr(gd[name], gref[name]) <= 6e-2, (name, relerr(gd[name], gref[name]))


def test_full_resolution_kernels_match_oracle():
    """A grid and batch large enough (256 x 256 x 4 pixels) for the
    full-resolution layers to take the LDS-tiled convolution (4 rows x 64
    pixels per block) and the weight gradients their per-wave and
    row-staged kernels: forward, loss and every layer's weight gradient
    against the float64 oracle."""
    net, flat, x, t = setup(256, 4, 5)
    y = net.forward(torch.from_numpy(x).cuda())
    params = as_dict(flat, CH)
    yref, tape = ows.forward(params, x.astype(np.float64))
    assert relerr(y.cpu().numpy(), yref) <= 3e-2
    loss, g = net.gradient(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    lref = ows.loss(yref, t.astype(np.float64))
    gref = ows.backward(params, tape, t.astype(np.float64))
    assert abs(loss - lref) <= 3e-2 * lref
    gd = as_dict(g, CH)
    for name in rp.WS_LAYERS:
        assert relerr(gd[name], gref[name]) <= 6e-2, (name, relerr(gd[name], gref[name]))
    # the partial sums are added in a fixed order: the same inputs give the
    # same loss and gradient bit for bit
    loss2, g2 = net.gradient(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    assert loss2 == loss and np.array_equal(g2, g)


@pytest.mark.parametrize("grid,B,channels", [(48, 2, (40, 48, 56, 64, 64)),
                                              (80, 2, (12, 36, 64, 40, 40))])
def test_wide_channels_and_ragged_tiles_match_oracle(grid, B, channels):
    """Channel widths that pad to 64 (and to 32 next to 64), on grids whose
    levels (48 .. 3, 80 .. 5) leave partial 64-pixel tiles, partial 4-row
    tiles and widths that are no multiple of 4: forward, loss and every
    layer's weight gradient against the float64 oracle."""
    net, flat, x, t = setup(grid, B, 7, channels)
    params = as_dict(flat, channels)
    yref, tape = ows.forward(params, x.astype(np.float64))
    y = net.forward(torch.from_numpy(x).cuda())
    assert relerr(y.cpu().numpy(), yref) <= 3e-2
    loss, g = net.gradient(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    lref = ows.loss(yref, t.astype(np.float64))
    gref = ows.backward(params, tape, t.astype(np.float64))
    assert abs(loss - lref) <= 3e-2 * lref
    gd = as_dict(g, channels)
    for name in rp.WS_LAYERS:
        assert relerr(gd[name], gref[name]) <= 6e-2, (name, relerr(gd[name], gref[name]))


def test_adam_first_step_and_determinism():
    """Adam's first step moves every weight by -lr g / (|g| + eps) (its
    bias-corrected moments are g and g^2), with g the network's own
    gradient; two identical runs give identical weights."""
    runs = []
    for rep in range(2):
        net, flat, x, t = setup(32, 2, 3)
        xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
        _, g = net.gradient(xd, td)
        net.adam(1e-3)
        w1 = net.get_weights()
        step = (w1.astype(np.float64) - flat) / 1e-3
        want = -g / (np.abs(g.astype(np.float64)) + 1e-8)
        assert np.abs(step - want).max() <= 2e-3
        for _ in range(3):
            net.train_step(xd, td, 1e-3)
        runs.append(net.get_weights())
    assert np.array_equal(runs[0], runs[1])


def test_training_reduces_the_loss():
    """Fitting a fixed linear map of the input (k^2 u ~ -f for a source that
    does not radiate): forty Adam steps cut the loss several times."""
    net, flat, x, _ = setup(32, 4, 4)
    t = (-x).copy()
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    l0, _ = net.gradient(xd, td, want_grad=False)
    for _ in range(40):
        net.train_step(xd, td, 3e-3)
    l1, _ = net.gradient(xd, td, want_grad=False)
    assert l1 < 0.3 * l0, (l0, l1)


def small_problem():
    # grid = n_int = 32 (divisible by 16)
    return Problem(k=16.0, n_int=32, G=4, Px=2, Py=2, delta=4, kappa=4, sigma=160.0)


def setup_handle(pb):
    o = rp.default_opts(sigma=pb.sigma, global_pml=pb.G, precision=rp.RAS_FP64)
    return rp.ras_pml_setup(pb.k, 1.0 / pb.n_int, (pb.n_int, pb.n_int), (pb.Px, pb.Py), pb.delta,
                            pb.kappa, o)


def test_grid_sample_is_the_interior_nodes():
    pb = small_problem()
    H = setup_handle(pb)
    assert H.grid_side() == 32
    v = inputs.random_vector(pb.ndof, 5)
    got = rp.ras_pml_grid_sample(H, torch.from_numpy(v).cuda(), 3.0).cpu().numpy()
    gx, gy = np.meshgrid(np.arange(32), np.arange(32), indexing="xy")
    idx = geometry.global_index(pb, pb.G + gx.ravel(), pb.G + gy.ravel())
    want = np.stack([(3.0 * v[idx]).real, (3.0 * v[idx]).imag], -1).astype(np.float32)
    assert np.array_equal(got.reshape(-1, 2), want)


def test_warm_start_guess_and_fallback():
    pb = small_problem()
    H = setup_handle(pb)
    R = ras.RasPml(pb)
    f = inputs.gaussian(pb.n_int, pb.G, [(0.4, 0.55)], [1.0], 0.08)
    b = fem.rhs(R.M1, f)
    fd, bd = torch.from_numpy(f).cuda(), torch.from_numpy(b).cuda()
    x0 = torch.ones_like(fd)
    # the guess the network makes, on the interior nodes, over k^2
    net = rp.WSNet(32, CH, 1)
    flat = inputs.ws_init_weights(rp.ws_shapes(CH), 6, gain=0.05)
    net.set_weights(flat)
    used = rp.ras_pml_warm_start(H, net, fd, bd, x0)
    xs = x0.cpu().numpy()
    gx, gy = np.meshgrid(np.arange(32), np.arange(32), indexing="xy")
    idx = geometry.global_index(pb, pb.G + gx.ravel(), pb.G + gy.ravel())
    fg = np.stack([f[idx].real, f[idx].imag], -1).reshape(1, 32, 32, 2)
    yref, _ = ows.forward(as_dict(flat, CH), fg)
    guess = (yref[0, :, :, 0] + 1j * yref[0, :, :, 1]).ravel() / pb.k ** 2
    if used:
        assert relerr(xs[idx], guess) <= 3e-2
        mask = np.ones(pb.ndof, bool)
        mask[idx] = False
        assert np.all(xs[mask] == 0)
        assert np.linalg.norm(b - R.A @ xs) <= np.linalg.norm(b)
    else:
        assert np.all(xs == 0)
    # a guess far too large is rejected: x0 = 0
    net.set_weights(inputs.ws_init_weights(rp.ws_shapes(CH), 6, gain=50.0))
    x0 = torch.ones_like(fd)
    assert not rp.ras_pml_warm_start(H, net, fd, bd, x0)
    assert torch.count_nonzero(x0) == 0
    # zero weights: the guess is zero and is kept (its residual is ||b||)
    net.set_weights(np.zeros(net.nweights, np.float32))
    x0 = torch.ones_like(fd)
    assert rp.ras_pml_warm_start(H, net, fd, bd, x0)
    assert torch.count_nonzero(x0) == 0
    # the source scale is divided out before the network and multiplied back
    # after it: with fscale = 2 the guess is 2 * network(f / 2) / k^2
    net.set_weights(flat)
    x2 = torch.zeros_like(fd)
    rp.ras_pml_warm_start(H, net, fd, bd, x2, fscale=2.0)
    y2, _ = ows.forward(as_dict(flat, CH), fg / 2.0)
    guess2 = 2.0 * (y2[0, :, :, 0] + 1j * y2[0, :, :, 1]).ravel() / pb.k ** 2
    x2h = x2.cpu().numpy()
    if np.any(x2h != 0):
        assert relerr(x2h[idx], guess2) <= 3e-2
    with pytest.raises(rp.RasPmlError):
        rp.ras_pml_warm_start(H, net, fd, bd, x2, fscale=0.0)
    # GMRES from the guess converges to the same tolerance
    net.set_weights(flat)
    x0 = torch.zeros_like(fd)
    rp.ras_pml_warm_start(H, net, fd, bd, x0)
    rc, it, rr, _ = rp.gmres_solve(H, bd, x0, rtol=1e-8, restart=50, maxit=200)
    assert rc == rp.RAS_OK and np.linalg.norm(b - R.A @ x0.cpu().numpy()) <= 1e-8 * np.linalg.norm(b) * (1 + 1e-6)
