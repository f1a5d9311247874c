"""The curved no-slip wall around a disk (section 3-b) on the GPU: the sweep kernels bit for
bit against the reference kernels (the ghost fill is shared), both against the FP64 oracle,
and the decay rates of the 17 Stokes modes of Tables 2 and 3, measured with the library's
FP64 device projection, against the oracle's rates, the Bessel rates and the paper's.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import disk as D

pytestmark = pytest.mark.gpu

R, N = 29.9, 72
C = (N - 1) / 2
# the Tables 2-3 disk; an off-centre one in a ragged grid; the smallest radius allowed (a
# few fluid nodes); and one centred on a node
GEOMS = {"centred": (72, 72, C, C, R), "offset": (50, 41, 24.3, 19.8, 11.7), "tiny": (12, 12, 5.5, 5.5, 1.6),
         "node": (40, 40, 20.0, 19.0, 15.3)}
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "stokes_disk_tables.json")
NUS = {"0.05": 0.05, "1/sqrt108": 1.0 / math.sqrt(108.0)}


@pytest.fixture(scope="module")
def F():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1803_00437_amd as F

    F.load_library()
    return F


@pytest.fixture(scope="module")
def rules():
    return {k: D.disk_ghost_rules(*g) for k, g in GEOMS.items()}


def rel_l2(a, b):
    return math.sqrt(sum(float(np.sum((x - y) ** 2)) for x, y in zip(a, b)) / sum(float(np.sum(y * y)) for y in b))


def inside_noise(geom, seed, amp=1e-3):
    nx, ny, cx, cy, r = GEOMS[geom]
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    fluid = np.hypot(x - cx, y - cy) < r
    rng = np.random.default_rng(seed)
    return tuple(np.where(fluid, amp * rng.standard_normal((ny, nx)), 0.0) for _ in range(3))


def run(F, geom, init, steps, **kw):
    nx, ny, cx, cy, r = GEOMS[geom]
    sim = F.FdLbm(nx, ny, bc="disk", disk=(cx, cy, r), **kw)
    sim.set_state(*init)
    sim.step(steps)
    out = sim.get_state()
    sim.close()
    return out


@pytest.mark.parametrize("geom", list(GEOMS))
@pytest.mark.parametrize("dtype", ["f64", "f32", "f16", "f16sr"])
@pytest.mark.parametrize("scheme,stencil,forced", [("fd", 3, False), ("fd", 5, False), ("fd", 3, True),
                                                   ("fd", 5, True), ("lwacm", 3, False)])
def test_disk_sweep_equals_reference_bitwise(F, geom, dtype, scheme, stencil, forced):
    print(f"case disk sweep-vs-reference geom={geom} dtype={dtype} scheme={scheme} stencil={stencil} forced={forced}",
          flush=True)
    init = inside_noise(geom, seed=7)
    kw = dict(scheme=scheme, stencil=stencil, dtype=dtype, s_xx=O.rate_from_viscosity(0.05),
              force=(2e-6, -1e-6) if forced else (0.0, 0.0))
    a = run(F, geom, init, 40, kernel="reference", **kw)
    b = run(F, geom, init, 40, kernel="sweep", **kw)
    for u, v in zip(a, b):
        assert np.array_equal(u, v), float(np.max(np.abs(u - v)))


@pytest.mark.parametrize("geom", list(GEOMS))
@pytest.mark.parametrize("scheme", ["fd3", "fd5", "lwacm"])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_disk_matches_oracle(F, rules, geom, scheme, dtype, tol):
    """A Stokes mode plus noise (noise alone when the centre is a node), 200 steps, every
    node (fluid, ghost and rest) compared."""
    nx, ny, cx, cy, r = GEOMS[geom]
    nu, steps = 0.05, 200
    init = inside_noise(geom, seed=3, amp=2e-4)
    if geom != "node":
        k = W.disk_mode_wavenumber(2, 1, r)
        mode = W.disk_stokes_mode(nx, ny, cx, cy, r, 2, k, nu=nu)
        init = tuple(a + b for a, b in zip(mode, init))
    s_xx = O.rate_from_viscosity(nu)
    if scheme == "lwacm":
        got = run(F, geom, init, steps, scheme="lwacm", dtype=dtype, s_xx=s_xx)
        want = D.disk_run(*init, steps, rules=rules[geom], scheme="lwacm", s_xx=s_xx)
    else:
        st = int(scheme[2])
        got = run(F, geom, init, steps, scheme="fd", stencil=st, dtype=dtype, s_xx=s_xx, force=(1e-6, 0.0))
        want = D.disk_run(*init, steps, rules=rules[geom], stencil=st, s_xx=s_xx, fx=1e-6)
    err = rel_l2(got, want)
    print(f"  disk {geom} {scheme} {dtype}: rel L2 {err:.2e}")
    assert err <= tol


@pytest.mark.parametrize("geom", ["centred", "tiny"])
@pytest.mark.parametrize("forced", [False, True])
def test_disk_rest_nodes_set_by_the_caller_are_cleared(F, rules, geom, forced):
    """Noise on every node, the disk's outside included: the first step clears every rest
    node, later steps only the ring the step can reach (or every rest node again under a
    body force); FP64 against the oracle, which clears every rest node at every step,
    node by node, over 60 steps and again after a second set_state."""
    nx, ny, cx, cy, r = GEOMS[geom]
    rng = np.random.default_rng(11)
    init = tuple(1e-3 * rng.standard_normal((ny, nx)) for _ in range(3))
    force = (1e-6, -2e-6) if forced else (0.0, 0.0)
    s_xx = O.rate_from_viscosity(0.05)
    sim = F.FdLbm(nx, ny, bc="disk", disk=(cx, cy, r), stencil=5, dtype="f64", s_xx=s_xx, force=force)
    for rep in range(2):
        sim.set_state(*init)
        sim.step(60)
        got = sim.get_state()
        want = D.disk_run(*init, 60, rules=rules[geom], stencil=5, s_xx=s_xx, fx=force[0], fy=force[1])
        err = rel_l2(got, want)
        print(f"  disk {geom} forced={forced} set {rep}: rel L2 {err:.2e}")
        assert err <= 1e-12
        init = tuple(a[::-1, ::-1].copy() for a in init)
    sim.close()


def test_disk_f16_storage_error(F, rules):
    k = W.disk_mode_wavenumber(0, 2, R)
    init = W.disk_stokes_mode(N, N, C, C, R, 0, k, amp=0.01, nu=0.05)
    s_xx = O.rate_from_viscosity(0.05)
    got = run(F, "centred", init, 300, stencil=5, dtype="f16", s_xx=s_xx)
    want = D.disk_run(*init, 300, rules=rules["centred"], stencil=5, s_xx=s_xx)
    fl = rules["centred"]["fluid"]
    err = rel_l2([g[fl] for g in got], [w[fl] for w in want])
    print(f"  disk f16 rel L2 (fluid) {err:.2e}")
    assert err <= 5e-3


def table_modes():
    rows = json.load(open(GOLDEN))["rows"]
    return [(r, 0, r["l"]) if r["family"] == "singlet" else (r, r["l"], 1) for r in rows]


def device_rate(F, init, nu, gamma0, **kw):
    t1, t2 = D.decay_times(gamma0)
    sim = F.FdLbm(N, N, bc="disk", disk=(C, C, R), s_xx=O.rate_from_viscosity(nu), **kw)
    sim.set_state(*init)
    sim.set_mode(init[1], init[2])
    sim.step(t1)
    a1 = sim.mode_projection()
    sim.step(t2 - t1)
    a2 = sim.mode_projection()
    sim.close()
    return -math.log(a2 / a1) / (t2 - t1)


@pytest.mark.parametrize("stencil", [3, 5])
@pytest.mark.parametrize("nukey", list(NUS))
def test_stokes_mode_rates_tables_2_3(F, rules, stencil, nukey):
    """FP64 device rates of the 17 modes: equal to the oracle's to 1e-8 (relative), within
    2 % (3-point) or 0.3 % (5-point) of the paper's measured rates, and, 5-point, within
    0.6 % of nu a^2 / R^2; FP32 storage moves no rate by more than 1e-4."""
    nu = NUS[nukey]
    tol_paper = 0.02 if stencil == 3 else 0.003
    worst = 0.0
    for row, m, l in table_modes():
        k = W.disk_mode_wavenumber(m, l, R)
        init = W.disk_stokes_mode(N, N, C, C, R, m, k, nu=nu)
        g0 = nu * k * k
        got = device_rate(F, init, nu, g0, stencil=stencil, dtype="f64")
        want = D.disk_decay_rate(init, rules=rules["centred"], nu=nu, gamma0=g0, stencil=stencil)
        assert abs(got / want - 1) < 1e-8, (row, got, want)
        paper = row[f"fd{stencil}_nu_{nukey}"]
        ratio = (got / g0) / (1 + paper) - 1
        worst = max(worst, abs(ratio))
        assert abs(ratio) < tol_paper, (row, got / g0 - 1, paper)
        if stencil == 5:
            assert abs(got / g0 - 1) < 6e-3, (row, got / g0 - 1)
        if row["l"] in (1, 6):
            g32 = device_rate(F, init, nu, g0, stencil=stencil, dtype="f32")
            assert abs(g32 / got - 1) < 1e-4, (row, g32, got)
        print(f"  FD{stencil} nu={nukey} {row['family']} l={row['l']}: error {got / g0 - 1:+.5f} "
              f"(paper {paper:+.5f})")
    print(f"  FD{stencil} nu={nukey}: worst rate ratio to the paper {worst:.4f}")


@pytest.mark.parametrize("dtype", ["f32", "f16sr"])
def test_disk_autotune_leaves_the_run_unchanged(F, dtype):
    """fdlbm_autotune on a disk context times the step kernel on the current state without
    advancing it; the run that follows equals an untuned one bit for bit (every tile shape
    gives the same bits, and stochastic rounding draws from the step count, which tuning
    does not move)."""
    nx, ny, cx, cy, r = GEOMS["centred"]
    init = inside_noise("centred", seed=21)
    kw = dict(bc="disk", disk=(cx, cy, r), stencil=3, dtype=dtype, s_xx=O.rate_from_viscosity(0.05))
    out = []
    for tune in (False, True):
        sim = F.FdLbm(nx, ny, **kw)
        sim.set_state(*init)
        sim.step(5)
        if tune:
            sim.autotune(reps=3)
        sim.step(45)
        out.append(sim.get_state())
        sim.close()
    for u, v in zip(*out):
        assert np.array_equal(u, v)


# ------------------------------------------------- MRT D2Q9 in the disk (Tables 2-3) ----

LB_COLUMNS = {
    "bgk_nu_0.05": ("0.05", "bgk"), "lbe_q_nu_0.05": ("0.05", "quartic"),
    "bgk_nu_1/sqrt108": ("1/sqrt108", "bgk"), "lb_sq1.3_nu_1/sqrt108": ("1/sqrt108", 1.3),
    "lb_q_nu_1/sqrt108": ("1/sqrt108", "quartic"),
}


def lb_rates(nu, kind):
    s_xx = O.rate_from_viscosity(nu)
    if kind == "bgk":
        return dict(s_xx=s_xx, s_e=s_xx, s_q=s_xx, s_eps=s_xx)
    return dict(s_xx=s_xx, s_e=1.0, s_q=O.quartic_s_q(s_xx) if kind == "quartic" else kind, s_eps=1.0)


@pytest.fixture(scope="module")
def links():
    return {k: D.disk_links(*g) for k, g in GEOMS.items()}


def run_mrt(F, geom, init, steps, **kw):
    nx, ny, cx, cy, r = GEOMS[geom]
    sim = F.FdLbm(nx, ny, scheme="mrt", bc="disk", disk=(cx, cy, r), **kw)
    sim.set_state(*init)
    sim.step(steps)
    out = sim.get_populations()
    sim.close()
    return out


@pytest.mark.parametrize("geom", list(GEOMS))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("forced", [False, True])
def test_mrt_disk_sweep_equals_reference_bitwise(F, geom, dtype, forced):
    print(f"case mrt disk sweep-vs-reference geom={geom} dtype={dtype} forced={forced}", flush=True)
    init = inside_noise(geom, seed=17)
    kw = dict(dtype=dtype, force=(2e-6, -1e-6) if forced else (0.0, 0.0), **lb_rates(0.05, "quartic"))
    a = run_mrt(F, geom, init, 40, kernel="reference", **kw)
    b = run_mrt(F, geom, init, 40, kernel="sweep", **kw)
    assert np.array_equal(a, b), float(np.max(np.abs(a - b)))


@pytest.mark.parametrize("geom", list(GEOMS))
@pytest.mark.parametrize("kind", ["bgk", "quartic"])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_mrt_disk_matches_oracle(F, links, geom, kind, dtype, tol):
    """A Stokes mode plus noise (noise alone when the centre is a node), 200 steps under a
    small body force, every population of every node compared with the oracle's."""
    nx, ny, cx, cy, r = GEOMS[geom]
    nu, steps = 0.05, 200
    init = inside_noise(geom, seed=5, amp=2e-4)
    if geom != "node":
        k = W.disk_mode_wavenumber(2, 1, r)
        mode = W.disk_stokes_mode(nx, ny, cx, cy, r, 2, k, nu=nu)
        init = tuple(a + b for a, b in zip(mode, init))
    rates = lb_rates(nu, kind)
    got = run_mrt(F, geom, init, steps, dtype=dtype, force=(1e-6, 0.0), **rates)
    want = D.mrt_disk_run(O.mrt_init(*init), steps, links=links[geom], fx=1e-6, **rates)
    err = math.sqrt(float(np.sum((got - want) ** 2)) / float(np.sum(want ** 2)))
    print(f"  mrt disk {geom} {kind} {dtype}: rel L2 {err:.2e}")
    assert err <= tol


@pytest.mark.parametrize("geom", ["centred", "tiny"])
@pytest.mark.parametrize("forced", [False, True])
def test_mrt_disk_solid_nodes_set_by_the_caller_are_cleared(F, links, geom, forced):
    """Populations on every node, the solid outside included: the first step clears every
    solid node, later ones only the solid ring the links reach (or every solid node under a
    body force); FP64 populations equal the oracle's, which clears every solid node at every
    step, over 60 steps and again after a second set_populations."""
    nx, ny, cx, cy, r = GEOMS[geom]
    rng = np.random.default_rng(12)
    df = O.mrt_init(*(1e-3 * rng.standard_normal((ny, nx)) for _ in range(3)))
    force = (1e-6, -2e-6) if forced else (0.0, 0.0)
    rates = lb_rates(0.05, "quartic")
    sim = F.FdLbm(nx, ny, scheme="mrt", bc="disk", disk=(cx, cy, r), dtype="f64", force=force, **rates)
    for rep in range(2):
        sim.set_populations(df)
        sim.step(60)
        got = sim.get_populations()
        want = D.mrt_disk_run(df, 60, links=links[geom], fx=force[0], fy=force[1], **rates)
        err = math.sqrt(float(np.sum((got - want) ** 2)) / float(np.sum(want ** 2)))
        print(f"  mrt disk {geom} forced={forced} set {rep}: rel L2 {err:.2e}")
        assert err <= 1e-12
        df = df[:, ::-1, ::-1].copy()
    sim.close()


@pytest.mark.parametrize("col", list(LB_COLUMNS))
def test_lb_stokes_mode_rates_tables_2_3(F, links, col):
    """FP64 device rates of the 17 modes for the BGK and MRT columns of Tables 2 and 3: equal
    to the oracle's to 1e-8 (relative) and within 0.3 % of the paper's measured rates."""
    key, kind = LB_COLUMNS[col]
    nu = NUS[key]
    rates = lb_rates(nu, kind)
    worst = 0.0
    for row, m, l in table_modes():
        k = W.disk_mode_wavenumber(m, l, R)
        init = W.disk_stokes_mode(N, N, C, C, R, m, k, nu=nu)
        g0 = nu * k * k
        t1, t2 = D.decay_times(g0)
        sim = F.FdLbm(N, N, scheme="mrt", bc="disk", disk=(C, C, R), dtype="f64", **rates)
        sim.set_state(*init)
        sim.set_mode(np.where(links["centred"]["fluid"], init[1], 0.0), np.where(links["centred"]["fluid"], init[2], 0.0))
        sim.step(t1)
        a1 = sim.mode_projection()
        sim.step(t2 - t1)
        a2 = sim.mode_projection()
        sim.close()
        got = -math.log(a2 / a1) / (t2 - t1)
        want = D.mrt_disk_decay_rate(init, links=links["centred"], nu=nu, gamma0=g0, **rates)
        assert abs(got / want - 1) < 1e-8, (row, got, want)
        ratio = (got / g0) / (1 + row[col]) - 1
        worst = max(worst, abs(ratio))
        assert abs(ratio) < 3e-3, (row, got / g0 - 1, row[col])
        print(f"  {col} {row['family']} l={row['l']}: error {got / g0 - 1:+.5f} (paper {row[col]:+.5f})")
    print(f"  {col}: worst rate ratio to the paper {worst:.4f}")
