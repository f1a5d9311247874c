"""Host-side checks of the C ABI (no GPU): the library loads, exports every function that
include/fdlbm.h and include/fdlbm3d.h declare, and rejects invalid parameters before touching
a device."""
import ctypes
import os
import re

import pytest

import paper_1803_00437_amd as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("fdlbm.h", "fdlbm3d.h")]


def declared_functions():
    names = []
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_every_header_is_covered():
    assert sorted(os.listdir(os.path.join(ROOT, "include"))) == sorted(os.path.basename(h) for h in HEADERS)


def test_library_loads_and_exports_every_declared_function():
    lib = F.load_library()
    names = declared_functions()
    assert "fdlbm_step" in names and "mrt_step" in names and "fdlbm_diagnostics" in names
    assert "fdlbm3d_step" in names and "fdlbm3d_create" in names and "fdlbm3d_autotune" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(F.EXPORTED) == names


def test_params_struct_layout_matches_header():
    # 6 int32, 4 doubles, int32 (+pad), 2 doubles, 4 int32, 4 doubles
    assert ctypes.sizeof(F.Params) == 6 * 4 + 4 * 8 + 8 + 2 * 8 + 4 * 4 + 4 * 8
    assert F.Params.wall_xi.offset == 96
    assert F.Params.disk_r.offset == 120
    assert ctypes.sizeof(F.Diag) == 8 * 8


def good(**kw):
    base = dict(nx=64, ny=48, scheme="fd", stencil=3, bc="periodic", dtype="f32", s_xx=1.5, s_e=1.0)
    base.update(kw)
    return F.make_params(**base)


def test_workspace_bytes():
    sb, cb = F.fdlbm_workspace_bytes(good())
    assert sb >= 3 * 64 * 48 * 4 and sb % 256 == 0 and cb > 0
    sb64, _ = F.fdlbm_workspace_bytes(good(dtype="f64"))
    sb16, _ = F.fdlbm_workspace_bytes(good(dtype="f16"))
    assert sb64 >= 3 * 64 * 48 * 8 and sb16 >= 3 * 64 * 48 * 2 and sb16 < sb
    sbm, _ = F.fdlbm_workspace_bytes(good(scheme="mrt", s_q=1.2, s_eps=1.0))
    assert sbm >= 9 * 64 * 48 * 4


@pytest.mark.parametrize("bad", [
    dict(nx=4), dict(ny=2), dict(ny=6), dict(stencil=9), dict(stencil=4), dict(s_xx=2.0), dict(s_xx=0.0),
    dict(s_e=-1.0), dict(s_xx=float("nan")), dict(scheme="mrt", dtype="f16", s_q=1.0),
    dict(scheme="mrt", dtype="f16sr", s_q=1.0),
    dict(scheme="mrt", s_q=2.5), dict(scheme="mrt", s_eps=0.0), dict(force=(float("inf"), 0.0)),
])
def test_invalid_parameters_are_rejected(bad):
    with pytest.raises(F.FdlbmError) as e:
        F.fdlbm_workspace_bytes(good(**bad))
    assert e.value.code == F.FDLBM_EINVAL


@pytest.mark.parametrize("scheme", ["fd", "mrt"])
def test_tile_rows_are_bounded(scheme):
    """A tile taller than 1024 rows is rejected before any launch arithmetic (2^30 rows would
    overflow the block count), for the FD-LBM and MRT sweep kernels alike."""
    kw = dict(scheme=scheme, s_q=1.2) if scheme == "mrt" else dict(scheme=scheme)
    F.fdlbm_workspace_bytes(good(tile_rows=1024, **kw))
    for rows in (1025, 1 << 29, 1 << 30, (1 << 31) - 1, -1):
        with pytest.raises(F.FdlbmError) as e:
            F.fdlbm_workspace_bytes(good(tile_rows=rows, **kw))
        assert e.value.code == F.FDLBM_EINVAL


def test_set_step_count_rejects_null_and_negative():
    lib = F.load_library()
    assert lib.fdlbm_set_step_count(None, 5) == F.FDLBM_EINVAL
    assert lib.fdlbm_step_count(None) == -1


def test_wall_distance_is_checked_with_walls_only():
    """wall_xi: 0 selects 1/2, (0, 1] is accepted, other values are rejected with walls and
    ignored without them; both MRT kernels take any distance."""
    for xi in (0.0, 0.1, 0.5, 1.0):
        F.fdlbm_workspace_bytes(good(bc="walls", wall_xi=xi))
        F.fdlbm_workspace_bytes(good(bc="walls", wall_xi=xi, scheme="mrt", quartic=True))
    F.fdlbm_workspace_bytes(good(wall_xi=-3.0))
    for bad in (dict(wall_xi=-0.1), dict(wall_xi=1.5), dict(wall_xi=float("nan"))):
        with pytest.raises(F.FdlbmError) as e:
            F.fdlbm_workspace_bytes(good(bc="walls", **bad))
        assert e.value.code == F.FDLBM_EINVAL
    for xi in (0.3, 0.5, 0.8):
        F.fdlbm_workspace_bytes(good(bc="walls", wall_xi=xi, scheme="mrt", quartic=True, kernel="sweep"))


def test_lwacm_is_periodic_without_force():
    """Section 1-b defines the LW-ACM step on a periodic grid without body force; its stencil
    and s_e are not used."""
    F.fdlbm_workspace_bytes(good(scheme="lwacm", stencil=9, s_e=1.7))
    F.fdlbm_workspace_bytes(good(scheme="lwacm", dtype="f16", lane_cols=1, kernel="sweep"))
    for bad in (dict(bc="walls"), dict(force=(1e-5, 0.0)), dict(lane_cols=3)):
        with pytest.raises(F.FdlbmError) as e:
            F.fdlbm_workspace_bytes(good(scheme="lwacm", **bad))
        assert e.value.code == F.FDLBM_EINVAL


def test_walls_allow_small_ny_and_quartic_needs_no_s_q():
    F.fdlbm_workspace_bytes(good(bc="walls", ny=4))
    F.fdlbm_workspace_bytes(good(scheme="mrt", quartic=True, s_q=0.0))


def test_create_rejects_bad_buffers_without_a_device():
    lib = F.load_library()
    p = good()
    ctx = ctypes.c_void_p()
    # NULL buffers, identical ping-pong buffers and misaligned buffers are refused before any HIP call
    assert lib.fdlbm_create(ctypes.byref(p), None, None, None, 0, None, ctypes.byref(ctx)) == F.FDLBM_EINVAL
    assert lib.fdlbm_create(ctypes.byref(p), 4096, 4096, 8192, 1 << 30, None, ctypes.byref(ctx)) == F.FDLBM_EINVAL
    assert lib.fdlbm_create(ctypes.byref(p), 4100, 8192, 16384, 1 << 30, None, ctypes.byref(ctx)) == F.FDLBM_EINVAL
    assert lib.fdlbm_create(ctypes.byref(p), 4096, 8192, 16384, 16, None, ctypes.byref(ctx)) == F.FDLBM_ENOMEM


def test_null_context_is_rejected():
    lib = F.load_library()
    assert lib.fdlbm_step(None, 1) == F.FDLBM_EINVAL
    assert lib.mrt_step(None, 1) == F.FDLBM_EINVAL
    assert lib.lwacm_step(None, 1) == F.FDLBM_EINVAL
    assert lib.fdlbm_step_count(None) == -1


def test_rate_helpers_match_section_1a_and_3b():
    assert abs(F.fdlbm_rate_from_viscosity(0.02) - 1 / (0.5 + 0.06)) < 1e-15
    s_xx = F.fdlbm_rate_from_viscosity(1 / 108 ** 0.5)
    s_q = F.fdlbm_quartic_s_q(s_xx)
    assert abs((1 / s_xx - 0.5) * (1 / s_q - 0.5) - 1 / 6) < 1e-14
    assert abs(s_q - 0.9282) < 0.5e-4


def test_strerror():
    lib = F.load_library()
    for code in (0, -1, -2, -3, -4):
        assert lib.fdlbm_strerror(code)


def test_batch_workspace_and_validation():
    specs = [(33, 40, 1.6, 1.0), (64, 64, 1.2, 1.1)]
    sb, cb = F.fdlbm_batch_workspace_bytes(specs, "f32", 10)
    assert sb >= 3 * (33 * 40 + 64 * 64) * 4 and sb % 256 == 0 and cb > 0
    for bad in ([(4, 40, 1.6, 1.0)], [(33, 40, 2.0, 1.0)], [(33, 40, 1.6, 0.0)]):
        with pytest.raises(F.FdlbmError) as e:
            F.fdlbm_batch_workspace_bytes(bad, "f32", 10)
        assert e.value.code == F.FDLBM_EINVAL
    with pytest.raises(F.FdlbmError):
        F.fdlbm_batch_workspace_bytes(specs, "f32", -1)


def test_autotune_rejects_bad_arguments_without_a_device():
    lib = F.load_library()
    assert lib.fdlbm_autotune(None, 5, None, None, None) == F.FDLBM_EINVAL
    assert lib.fdlbm_batch_autotune(None, 5, None, None) == F.FDLBM_EINVAL


def disk(**kw):
    base = dict(nx=72, ny=72, bc="disk", disk=(35.5, 35.5, 29.9), s_xx=1.5)
    base.update(kw)
    return good(**base)


def test_disk_table_size_matches_the_oracle_ghost_count():
    """The scratch buffer grows by the ghost-node table: two int32 and three doubles per
    ghost node, two int32 per row, and one int32 per ring node (the rest nodes within the
    step's reach of a fluid or ghost node, across the periodic edges), each array 256-byte
    aligned.  The counts are the ones the oracle's geometry gives (section 3-b), so the
    host-side table builder and the oracle agree on which nodes are ghosts."""
    import numpy as np
    from oracle import disk as D

    def a256(x):
        return (x + 255) // 256 * 256

    for (nx, ny, cx, cy, r) in ((72, 72, 35.5, 35.5, 29.9), (50, 41, 24.3, 19.8, 11.7), (20, 20, 9.0, 9.5, 2.2),
                                (12, 12, 5.5, 5.5, 1.6)):
        rules = D.disk_ghost_rules(nx, ny, cx, cy, r)
        ng = rules["j"].size
        active = ~rules["rest"]
        near = np.zeros_like(active)
        for dy in range(-3, 4):
            for dx in range(-3, 4):
                near |= np.roll(np.roll(active, dy, 0), dx, 1)
        nr = int(np.count_nonzero(near & rules["rest"]))
        _, base = F.fdlbm_workspace_bytes(good(nx=nx, ny=ny))
        _, cb = F.fdlbm_workspace_bytes(good(nx=nx, ny=ny, bc="disk", disk=(cx, cy, r)))
        assert cb - base == 2 * a256(4 * ng) + a256(24 * ng) + a256(8 * ny) + a256(4 * nr), (nx, ny, cx, cy, r)


@pytest.mark.parametrize("bad", [
    dict(disk=(35.5, 35.5, 34.0)),          # reaches past the edge (needs cx - r >= 2)
    dict(disk=(35.5, 35.5, 33.6)),          # cx + r > nx - 3
    dict(disk=(10.0, 35.5, 9.0)),
    dict(disk=(35.5, 35.5, 1.5)),           # the depth-3/2 sample needs r > 3/2
    dict(disk=(35.5, 35.5, 0.0)),
    dict(disk=(float("nan"), 35.5, 10.0)),
    dict(disk=(35.5, 35.5, float("inf"))),
    dict(scheme="mrt", quartic=True, dtype="f16"),  # MRT stores FP64 or FP32 populations
    dict(scheme="lwacm", force=(1e-6, 0.0)),
])
def test_disk_parameters_are_checked(bad):
    with pytest.raises(F.FdlbmError) as e:
        F.fdlbm_workspace_bytes(disk(**bad))
    assert e.value.code == F.FDLBM_EINVAL


def test_mrt_disk_table_size_matches_the_oracle_link_count():
    """MRT in the disk: the scratch buffer grows by the boundary-link table (node, direction
    and q per link), the solid nodes the links reach, and the fluid span of each row; the
    link count is the oracle's (every fluid node with a solid neighbour, per direction)."""
    import numpy as np
    from oracle import disk as D

    def a256(x):
        return (x + 255) // 256 * 256

    for (nx, ny, cx, cy, r) in ((72, 72, 35.5, 35.5, 29.9), (50, 41, 24.3, 19.8, 11.7), (12, 12, 5.5, 5.5, 1.6)):
        links = D.disk_links(nx, ny, cx, cy, r)
        ex, ey = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1]), np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
        nl = links["k"].size
        nsr = len({(j + ey[k], i + ex[k]) for j, i, k in zip(links["j"], links["i"], links["k"])})
        kw = dict(nx=nx, ny=ny, scheme="mrt", quartic=True)
        _, base = F.fdlbm_workspace_bytes(good(**kw))
        _, cb = F.fdlbm_workspace_bytes(good(bc="disk", disk=(cx, cy, r), **kw))
        assert cb - base == 2 * a256(4 * nl) + a256(8 * nl) + a256(4 * nsr) + a256(8 * ny), (nx, ny, cx, cy, r)


def test_disk_accepts_every_fd_variant():
    for kw in (dict(), dict(stencil=5), dict(dtype="f64"), dict(dtype="f16"), dict(scheme="lwacm"),
               dict(force=(1e-6, 0.0)), dict(kernel="reference"), dict(kernel="sweep", lane_cols=2),
               dict(disk=(35.5, 35.5, 1.6)), dict(disk=(31.9, 31.9, 29.9)),
               dict(scheme="mrt", quartic=True), dict(scheme="mrt", s_q=1.3, dtype="f64", kernel="reference"),
               dict(scheme="mrt", quartic=True, force=(1e-6, 0.0))):
        F.fdlbm_workspace_bytes(disk(**kw))


def test_stochastic_rounding_storage_is_for_single_fd_grids():
    """FDLBM_F16DEV_SR: FD-LBM and LW-ACM single grids (any stencil, walls, disk); the batch
    and MRT reject it."""
    for kw in (dict(), dict(stencil=5), dict(scheme="lwacm"), dict(bc="walls"),
               dict(nx=72, ny=72, bc="disk", disk=(35.5, 35.5, 29.9))):
        sb, _ = F.fdlbm_workspace_bytes(good(dtype="f16sr", **kw))
        assert sb == F.fdlbm_workspace_bytes(good(dtype="f16", **kw))[0]
    lib = F.load_library()
    inst = (F.Instance * 1)(F.Instance(64, 64, 1.5, 1.0))
    sb, cb = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.fdlbm_batch_workspace_bytes(inst, 1, F.DTYPE["f16sr"], 4, ctypes.byref(sb),
                                           ctypes.byref(cb)) == F.FDLBM_EINVAL
    assert lib.fdlbm_batch_workspace_bytes(inst, 1, F.DTYPE["f16"], 4, ctypes.byref(sb),
                                           ctypes.byref(cb)) == F.FDLBM_OK


def test_header_is_c99_and_links(tmp_path):
    """include/fdlbm.h compiles as C99 with warnings as errors (no C++ in the declarations), every function
    it declares links against libfdlbm.so, and a plain C caller gets the same workspace
    sizes and error codes as the Python binding (no device is touched)."""
    import shutil
    import subprocess

    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    names = declared_functions()
    src = tmp_path / "caller.c"
    refs = "\n".join(f"    (void *)&{n}," for n in names)
    src.write_text(f"""
#include <stdio.h>
#include <string.h>
#include "fdlbm.h"
#include "fdlbm3d.h"
static void *const every_function[] = {{
{refs}
}};
int main(void)
{{
    fdlbm_params p;
    size_t sb = 0, cb = 0;
    memset(&p, 0, sizeof p);
    p.nx = 64; p.ny = 48; p.scheme = FDLBM_SCHEME_FD; p.stencil = 3; p.bc = FDLBM_BC_PERIODIC;
    p.dtype = FDLBM_F32; p.s_xx = 1.5; p.s_e = 1.0;
    int rc = fdlbm_workspace_bytes(&p, &sb, &cb);
    p.stencil = 9;
    int bad = fdlbm_workspace_bytes(&p, &sb, &cb);
    printf("%d %zu %zu %d %d %s\\n", rc, sb, cb, bad, (int)(sizeof every_function / sizeof every_function[0]),
           fdlbm_strerror(bad));
    return 0;
}}
""")
    lib_dir = os.path.dirname(F.LIB_PATH)
    exe = tmp_path / "caller"
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", f"-I{os.path.join(ROOT, 'include')}",
           str(src), "-o", str(exe), f"-L{lib_dir}", "-lfdlbm", f"-Wl,-rpath,{lib_dir}",
           "-Wl,--allow-shlib-undefined"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    rc, sb, cb, bad, count = (int(x) for x in r.stdout.split()[:5])
    want_sb, want_cb = F.fdlbm_workspace_bytes(good())
    assert (rc, sb, cb, bad, count) == (0, want_sb, want_cb, F.FDLBM_EINVAL, len(names))
    assert "invalid argument" in r.stdout


def test_params3d_struct_layout_matches_header():
    # 4 int32, 2 doubles, 3 int32 (+pad)
    assert ctypes.sizeof(F.Params3D) == 4 * 4 + 2 * 8 + 3 * 4 + 4
    assert F.Params3D.s_nu.offset == 16 and F.Params3D.kernel.offset == 32
    assert ctypes.sizeof(F.Diag3D) == 7 * 8


def good3(**kw):
    base = dict(nx=64, ny=40, nz=24, dtype="f32", s_nu=1.5, s_e=1.2)
    base.update(kw)
    return F.make_params3d(**base)


def test_workspace_bytes_3d():
    n = 64 * 40 * 24
    sb, cb = F.fdlbm3d_workspace_bytes(good3())
    assert sb >= 4 * n * 4 and sb % 256 == 0 and cb >= 4 * n * 8
    sb64, _ = F.fdlbm3d_workspace_bytes(good3(dtype="f64"))
    assert sb64 >= 4 * n * 8
    _, cref = F.fdlbm3d_workspace_bytes(good3(kernel="reference"))
    assert cref >= cb + 18 * n * 4


@pytest.mark.parametrize("bad", [
    dict(nx=2), dict(ny=2), dict(nz=2), dict(nx=(1 << 20) + 1), dict(s_nu=2.0), dict(s_nu=0.0), dict(s_e=-1.0),
    dict(s_e=float("nan")), dict(tile_rows=4), dict(tile_rows=14), dict(tile_rows=-1), dict(tile_planes=-1),
    dict(tile_planes=4097), dict(nx=1 << 20, ny=1 << 20, nz=3), dict(nx=1 << 15, ny=1 << 14, nz=3),
    dict(nx=1 << 14, ny=1 << 14, nz=3, dtype="f64"),
])
def test_invalid_parameters_3d_are_rejected(bad):
    with pytest.raises(F.FdlbmError) as e:
        F.fdlbm3d_workspace_bytes(good3(**bad))
    assert e.value.code == F.FDLBM_EINVAL


def test_largest_3d_plane_is_accepted():
    """One plane just below 2^31 bytes is accepted (2^29 - 2^14 FP32 nodes, half of that in FP64)."""
    F.fdlbm3d_workspace_bytes(good3(nx=1 << 15, ny=(1 << 14) - 1, nz=3))
    F.fdlbm3d_workspace_bytes(good3(nx=1 << 14, ny=(1 << 14) - 1, nz=3, dtype="f64"))


def test_params3d_rejects_other_dtypes():
    for d in ("f16", "f16sr"):
        with pytest.raises(ValueError):
            good3(dtype=d)
    lib = F.load_library()
    p = good3()
    p.dtype = F.DTYPE["f16"]
    sb, cb = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.fdlbm3d_workspace_bytes(ctypes.byref(p), ctypes.byref(sb), ctypes.byref(cb)) == F.FDLBM_EINVAL


def test_product_never_reaches_the_oracle():
    """The library and its binding share nothing with the oracle: no source under the package
    names it, and the oracle names nothing of the package (only tests, smoke() and the CPU
    baseline of bench.py use the oracle)."""
    pkg = os.path.join(ROOT, "paper_1803_00437_amd")
    for dirpath, _, files in os.walk(pkg):
        if "_build" in dirpath or "__pycache__" in dirpath:
            continue
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text, os.path.join(dirpath, f)
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c")):
            text = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_1803_00437_amd" not in text and "fdlbm.h" not in text, f
