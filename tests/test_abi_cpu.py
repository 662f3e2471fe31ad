"""CPU tests of the C ABI: the library loads, exports every declared symbol,
and its host-only planning (validation, covering, descriptors) matches the
oracle's reading of the paper.  No compute call touches a GPU here."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2602_00735_amd as rp
from oracle import geometry
from oracle.geometry import BC_DRCH, BC_IMP, Problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ras_pml.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(rp.LIB_PATH):
        from paper_2602_00735_amd import build
        build.build()
    return rp.lib()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ \*]*?\b([a-z_][a-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("ras_pml_setup", "ras_pml_apply", "gmres_solve", "ras_pml_destroy",
                 "ras_pml_plan", "ras_pml_spmv", "ras_pml_rhs"):
        assert must in names


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    bound = {s[0] for s in rp.SYMBOLS}
    assert set(names) == bound


def test_device_memory_cache_calls_need_no_device(L):
    rp.ras_pml_set_cache_limit(1 << 30)
    assert rp.ras_pml_cache_info() == (0, 0)
    assert rp.ras_pml_empty_cache() == 0
    rp.ras_pml_set_cache_limit(-1)


def test_strerror(L):
    for s in range(9):
        assert rp.ras_pml_strerror(s)
    assert rp.ras_pml_strerror(99) == "unknown status"


@pytest.mark.parametrize("args,status", [
    (dict(k=-1.0), rp.RAS_EINVAL),
    (dict(k=float("nan")), rp.RAS_EINVAL),
    (dict(h=1.0 / 41), rp.RAS_EINVAL),            # grid * h != 1
    (dict(grid=(40, 39)), rp.RAS_EINVAL),
    (dict(subdomains=(0, 2)), rp.RAS_EINVAL),
    (dict(overlap=-2), rp.RAS_EINVAL),            # -1 is RAS_WIDTH_RULE
    (dict(pml_width=-3), rp.RAS_EINVAL),
    (dict(subdomains=(1, 1), grid=(500, 500), h=1 / 500), rp.RAS_ENOTSUP),   # band too wide
])
def test_plan_rejects_bad_parameters(L, args, status):
    kw = dict(k=20.0, h=1 / 40, grid=(40, 40), subdomains=(2, 2), overlap=6, pml_width=6)
    kw.update(args)
    with pytest.raises(rp.RasPmlError) as e:
        rp.ras_pml_plan(kw["k"], kw["h"], kw["grid"], kw["subdomains"], kw["overlap"],
                        kw["pml_width"], rp.default_opts(global_pml=4))
    assert e.value.status == status


def test_wide_band_columns_are_multiples_of_64(L):
    """Bands above 127 take the wide kernels: W = n_fast + 2 rounded up to a
    multiple of 64, up to 448 (Section 4's own subdomains, 300-cell cores
    with their overlap and PML, have n_fast of about 330..390)."""
    o = rp.default_opts(global_pml=6)
    for n_int, nf, W in ((115, 126, 128), (116, 127, 192), (194, 205, 256), (254, 265, 320),
                         (340, 351, 384), (370, 381, 384), (371, 382, 384), (372, 383, 448),
                         (434, 445, 448), (435, 446, 448)):
        d = rp.ras_pml_plan(40.0, 1 / n_int, (n_int, n_int), (1, 1), 0, 0, o)
        assert (d[0][1], d[0][2]) == (nf, W), (n_int, d[0][1], d[0][2])
    with pytest.raises(rp.RasPmlError) as e:
        rp.ras_pml_plan(40.0, 1 / 436, (436, 436), (1, 1), 0, 0, o)      # n_fast 447: W 449
    assert e.value.status == rp.RAS_ENOTSUP
    # the paper's Table 4 covering at k = 600 (16 subdomains, pml 16, ovlp 5,
    # global PML of three wavelengths): every band fits
    d = rp.ras_pml_plan(600.0, 1 / 1200, (1200, 1200), (4, 4), 5, 16, rp.default_opts(global_pml=38))
    assert max(x[2] for x in d) == 384 and min(x[2] for x in d) >= 192
    # Table 3's fixed PML of two wavelengths (25 cells) and overlap of two
    # thirds of one (8 cells) at k = 600: middle subdomains of band 387
    d = rp.ras_pml_plan(600.0, 1 / 1200, (1200, 1200), (4, 4), 8, 25, rp.default_opts(global_pml=37))
    assert max(x[1] for x in d) + 1 == 387 and max(x[2] for x in d) == 448


def test_setup_validation_runs_before_any_device_work(L):
    out = ctypes.c_void_p(123)
    rc = L.ras_pml_setup(20.0, 1 / 41, rp._i2((40, 40)), rp._i2((2, 2)), 6, 6, None, None,
                         ctypes.byref(out))
    assert rc == rp.RAS_EINVAL and out.value is None
    assert b"grid * h" in L.ras_pml_plan_error()
    o = rp.default_opts(bc=7)
    rc = L.ras_pml_setup(20.0, 1 / 40, rp._i2((40, 40)), rp._i2((2, 2)), 6, 6, ctypes.byref(o),
                         None, ctypes.byref(out))
    assert rc == rp.RAS_EINVAL


def test_boolean_pou_with_dirichlet_and_no_overlap_is_rejected(L):
    with pytest.raises(rp.RasPmlError) as e:
        rp.ras_pml_plan(10.0, 1 / 20, (20, 20), (2, 2), 0, 0,
                        rp.default_opts(bc=rp.RAS_BC_DRCH, pou=rp.RAS_POU_BOOLEAN, global_pml=2))
    assert e.value.status == rp.RAS_EINVAL


CASES = [
    ("k20", None),
    ("k160", None),
    ("k640", None),
    ("ragged", Problem(k=9.0, n_int=37, G=3, Px=3, Py=4, delta=3, kappa=2, sigma=90.0)),
    ("drch", Problem(k=9.0, n_int=37, G=3, Px=3, Py=4, delta=3, kappa=2, sigma=90.0, bc=BC_DRCH)),
    ("clip", Problem(k=9.0, n_int=30, G=2, Px=5, Py=5, delta=3, kappa=4, sigma=90.0)),
]


@pytest.mark.parametrize("name,pb", CASES)
def test_host_plan_matches_oracle_geometry(L, name, pb):
    if pb is None:
        pb = geometry.config_problem(name)
    opts = rp.default_opts(global_pml=pb.G, bc=pb.bc, sigma=pb.sigma)
    desc = rp.ras_pml_plan(pb.k, 1.0 / pb.n_int, (pb.n_int, pb.n_int), (pb.Px, pb.Py),
                           pb.delta, pb.kappa, opts)
    sds = geometry.subdomains(pb)
    assert len(desc) == len(sds)
    for d, sd in zip(desc, sds):
        assert d[0] == sd.n
        # factor column length: half-bandwidth + 1, rounded up to even
        assert d[1] == sd.n_fast and d[2] == sd.band + 1 + (sd.band + 1) % 2
        assert d[3] == int(sd.x_fast)
        assert (d[4], d[5], d[6], d[7]) == (sd.px.u_lo, sd.nx, sd.py.u_lo, sd.ny)
        assert (d[8], d[9]) == (sd.px.p, sd.py.p)
        assert (d[10], d[11], d[12], d[13]) == (sd.px.int_lo, sd.px.int_hi, sd.py.int_lo, sd.py.int_hi)
        assert (d[14], d[15], d[16], d[17]) == (sd.px.box_lo, sd.px.box_hi, sd.py.box_lo, sd.py.box_hi)
        flags = d[18]
        assert bool(flags & 1) == (sd.px.pml_lo > 0) and bool(flags & 2) == (sd.px.pml_hi > 0)
        assert bool(flags & 4) == (sd.py.pml_lo > 0) and bool(flags & 8) == (sd.py.pml_hi > 0)
        assert bool(flags & 16) == sd.px.imp_lo and bool(flags & 32) == sd.px.imp_hi
        assert bool(flags & 64) == sd.py.imp_lo and bool(flags & 128) == sd.py.imp_hi


def test_config_sizes_from_the_plan(L):
    """k = 640, h = 1/1280: 1305^2 = 1,703,025 unknowns (~1.7M), 32 x 32
    subdomains, interior extended sides of 92-93 cells."""
    pb = geometry.config_problem("k640")
    desc = rp.ras_pml_plan(640.0, 1 / 1280, (1280, 1280), (32, 32), pb.delta, pb.kappa,
                           rp.default_opts())
    assert len(desc) == 1024
    assert (pb.Nc - 1) ** 2 == 1703025
    sides = sorted(set(d[15] - d[14] for d in desc))
    assert sides[-1] in (92, 93) and 92 in sides
    assert max(d[2] for d in desc) <= 128


def _width_rows():
    rows = []
    for line in open(os.path.join(ROOT, "tests", "golden", "width_rule_tables.txt")):
        if line.strip() and not line.startswith("#"):
            rows.append(tuple(int(t) for t in line.split()))
    return rows


def test_width_rule_reproduces_the_paper_tables(L):
    """Section 3 (iii) widths through the C ABI against the printed Table 3/4
    columns (PML on the listed grid with C = 1/2, overlap at 12 points per
    wavelength with C = 1/6)."""
    for k, n, pml, ovlp in _width_rows():
        assert rp.ras_pml_width_rule(k, 1.0 / n, 0.5) == pml
        assert rp.ras_pml_width_rule(k, 2 * np.pi / k / 12, 1.0 / 6.0) == ovlp


def test_width_rule_matches_the_oracle_and_its_limit(L):
    rng = np.random.default_rng(5)
    for _ in range(400):
        k = float(rng.uniform(20.0, 20000.0))
        h = 1.0 / float(rng.integers(64, 40000))
        C = float(rng.choice([1 / 6, 1 / 4, 3 / 8, 1 / 2, 1.0]))
        assert rp.ras_pml_width_rule(k, h, C) == geometry.paper_width_cells(k, h, C)
    # k -> k0: l(k) -> 1/ln 2 from both sides, no 0/0
    for k in (150.0, 150.0 * (1 + 1e-9), 150.0 * (1 - 1e-9), 150.0 * (1 + 1e-4)):
        h = 1.0 / 3000
        want = geometry.paper_width_cells(150.0, h, 1.0)
        assert rp.ras_pml_width_rule(k, h, 1.0) == want
    for bad in ((0.0, 0.01, 0.5), (100.0, -1.0, 0.5), (100.0, 0.01, -0.5),
                (float("nan"), 0.01, 0.5), (100.0, 0.01, float("inf"))):
        with pytest.raises(ValueError):
            rp.ras_pml_width_rule(*bad)


def test_width_rule_as_a_setup_option(L):
    """RAS_WIDTH_RULE for overlap / pml_width plans exactly the subdomains of
    the explicit widths the rule gives (descriptor fields 20..22 carry the
    resolved delta, kappa and global PML)."""
    for k, n, P in ((80.0, 160, 4), (300.0, 600, 8), (640.0, 1280, 32)):
        h = 1.0 / n
        d = rp.ras_pml_width_rule(k, h, 1.0 / 6.0)
        kap = rp.ras_pml_width_rule(k, h, 0.5)
        o = rp.default_opts()
        a = rp.ras_pml_plan(k, h, (n, n), (P, P), rp.RAS_WIDTH_RULE, rp.RAS_WIDTH_RULE, o)
        b = rp.ras_pml_plan(k, h, (n, n), (P, P), d, kap, o)
        assert a == b
        assert all(row[20] == d and row[21] == kap and row[22] == kap for row in a)
        # other constants, explicit global PML
        o2 = rp.default_opts(width_c_kappa=3.0 / 8.0, width_k0=100.0, global_pml=7)
        c = rp.ras_pml_plan(k, h, (n, n), (P, P), 3, rp.RAS_WIDTH_RULE, o2)
        kap2 = rp.ras_pml_width_rule(k, h, 3.0 / 8.0, 100.0)
        assert all(row[20] == 3 and row[21] == kap2 and row[22] == 7 for row in c)
    o = rp.default_opts(width_c_delta=-1.0)
    with pytest.raises(Exception):
        rp.ras_pml_plan(80.0, 1 / 160, (160, 160), (4, 4), rp.RAS_WIDTH_RULE, 3, o)
    with pytest.raises(Exception):
        rp.ras_pml_plan(80.0, 1 / 160, (160, 160), (4, 4), -2, 3, rp.default_opts())


def test_shutdown_needs_no_device(L):
    """The exit hook's call: with nothing created it only returns."""
    assert L.ras_pml_shutdown() == rp.RAS_OK
    assert rp.ras_pml_cache_info() == (0, 0)
