"""C ABI checks that need no GPU: the library loads, exports every entry
point the header declares, and its host-side planning validates topology."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cfdhip.h")


def _lib():
    from paper_2012_02925_amd import capi
    if not os.path.exists(capi.LIB_PATH):
        from paper_2012_02925_amd import build
        build.build()
    return capi, capi.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cfd_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_and_library_exports_every_entry_point():
    capi, lib = _lib()
    names = declared_functions()
    assert len(names) >= 30
    for n in names:
        assert hasattr(lib, n), n
        assert n in capi.SIGNATURES, "binding missing for " + n


def _cfg(capi, dim=2, **kw):
    c = capi.CfdConfig()
    c.dim = dim
    c.gamma = 1.4
    c.limiter = 1
    c.muscl_eps = 1.0
    c.muscl_kappa = -1.0
    c.efix = 0.1
    c.rk_stages = 4
    c.dt_mode = 0
    c.cfl = 0.5
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def _ctx(capi, lib, **kw):
    ctx = ctypes.c_void_p()
    assert lib.cfd_create(ctypes.byref(_cfg(capi, **kw)), None, ctypes.byref(ctx)) == 0
    return ctx


def _add(capi, lib, ctx, ni, nj, nk=1, dim=2):
    if dim == 2:
        X = synth.cartesian_nodes_2d(ni, nj)
    else:
        X = synth.jittered_periodic_nodes_3d(ni, nj, nk, seed=0)
    X = np.ascontiguousarray(X)
    bid = ctypes.c_int()
    st = lib.cfd_add_block(ctx, ni, nj, nk, X.ctypes.data_as(capi._DP), ctypes.byref(bid))
    return st, bid.value


def _periodic(capi, lib, ctx, b, ni, nj):
    assert lib.cfd_connect(ctx, b, 0, capi.int2([0]), capi.int2([nj]), b, 1, capi.int2([0]), capi.int2([nj]), 0) == 0
    assert lib.cfd_connect(ctx, b, 2, capi.int2([0]), capi.int2([ni]), b, 3, capi.int2([0]), capi.int2([ni]), 0) == 0


def test_config_validation():
    capi, lib = _lib()
    ctx = ctypes.c_void_p()
    assert lib.cfd_create(ctypes.byref(_cfg(capi, dim=4)), None, ctypes.byref(ctx)) == -1
    assert lib.cfd_create(ctypes.byref(_cfg(capi, gamma=1.0)), None, ctypes.byref(ctx)) == -1
    assert lib.cfd_create(ctypes.byref(_cfg(capi, rk_stages=0)), None, ctypes.byref(ctx)) == -1
    assert lib.cfd_create(ctypes.byref(_cfg(capi, cfl=0.0)), None, ctypes.byref(ctx)) == -1
    assert lib.cfd_create(ctypes.byref(_cfg(capi, limiter=7)), None, ctypes.byref(ctx)) == -1
    assert lib.cfd_create(ctypes.byref(_cfg(capi, rk_scheme=2)), None, ctypes.byref(ctx)) == -1
    # the classical fourth-order method has exactly four stages
    assert lib.cfd_create(ctypes.byref(_cfg(capi, rk_scheme=capi.RK["classic4"], rk_stages=3)), None,
                          ctypes.byref(ctx)) == -1
    assert lib.cfd_create(ctypes.byref(_cfg(capi, rk_scheme=capi.RK["classic4"])), None, ctypes.byref(ctx)) == 0
    lib.cfd_destroy(ctx)


def test_flux_selection_validation():
    capi, lib = _lib()
    ctx = ctypes.c_void_p()
    assert lib.cfd_create(ctypes.byref(_cfg(capi, flux=3)), None, ctypes.byref(ctx)) == -1
    # the residual VJP is implemented for the Roe flux only
    ctx = _ctx(capi, lib, flux=capi.FLUX["vanleer_fvs"])
    _add(capi, lib, ctx, 8, 6)
    _periodic(capi, lib, ctx, 0, 8, 6)
    assert lib.cfd_enable_adjoint(ctx, 1) == 0
    n = ctypes.c_size_t()
    assert lib.cfd_finalize(ctx, ctypes.byref(n)) == -7
    assert b"Roe" in lib.cfd_last_error(ctx)
    lib.cfd_destroy(ctx)
    ctx = _ctx(capi, lib, flux=capi.FLUX["steger_warming"])
    _add(capi, lib, ctx, 8, 6)
    _periodic(capi, lib, ctx, 0, 8, 6)
    assert lib.cfd_finalize(ctx, ctypes.byref(n)) == 0
    lib.cfd_destroy(ctx)


def test_planning_and_workspace_size():
    capi, lib = _lib()
    ctx = _ctx(capi, lib)
    st, b = _add(capi, lib, ctx, 64, 48)
    assert st == 0 and b == 0
    _periodic(capi, lib, ctx, 0, 64, 48)
    n = ctypes.c_size_t()
    assert lib.cfd_finalize(ctx, ctypes.byref(n)) == 0
    assert n.value > 3 * 4 * 64 * 48 * 8
    v = ctypes.c_longlong()
    assert lib.cfd_query(ctx, capi.Q["ncells"], ctypes.byref(v)) == 0 and v.value == 64 * 48
    assert lib.cfd_query(ctx, capi.Q["ntransfers"], ctypes.byref(v)) == 0 and v.value == 4
    # 4 transfers x 2 layers x face length x 4 variables
    assert lib.cfd_query(ctx, capi.Q["exchange_doubles"], ctypes.byref(v)) == 0
    assert v.value == 4 * 2 * (48 + 48 + 64 + 64)
    lib.cfd_destroy(ctx)


def test_empty_context_cannot_finalize():
    capi, lib = _lib()
    ctx = _ctx(capi, lib)
    n = ctypes.c_size_t()
    assert lib.cfd_finalize(ctx, ctypes.byref(n)) == -2
    assert b"no blocks" in lib.cfd_last_error(ctx)
    lib.cfd_destroy(ctx)


def test_block_extent_and_range_errors():
    capi, lib = _lib()
    ctx = _ctx(capi, lib)
    assert _add(capi, lib, ctx, 1, 8)[0] == -1  # fewer than two cells
    assert _add(capi, lib, ctx, 8, 8)[0] == 0
    # range outside the face, bad face, bad kind
    assert lib.cfd_set_bc(ctx, 0, 0, capi.int2([0]), capi.int2([9]), 3, None, None) == -1
    assert lib.cfd_set_bc(ctx, 0, 5, capi.int2([0]), capi.int2([8]), 3, None, None) == -1
    assert lib.cfd_set_bc(ctx, 0, 0, capi.int2([0]), capi.int2([8]), 9, None, None) == -1
    # inflow needs positive density and pressure
    bad = (ctypes.c_double * 5)(-1.0, 1.0, 0.0, 1.0, 0.0)
    assert lib.cfd_set_bc(ctx, 0, 0, capi.int2([0]), capi.int2([8]), 2, ctypes.cast(bad, capi._DP), None) == -6
    lib.cfd_destroy(ctx)


def test_characteristic_bc_parameter_validation():
    capi, lib = _lib()
    ctx = _ctx(capi, lib)
    _add(capi, lib, ctx, 8, 6)
    K = capi.BC
    r = (capi.int2([0]), capi.int2([6]))
    rj = (capi.int2([0]), capi.int2([8]))

    def arr(*v):
        return ctypes.cast((ctypes.c_double * 5)(*(list(v) + [0.0] * (5 - len(v)))), capi._DP)

    # parameters are required, finite and positive where they are densities or pressures
    assert lib.cfd_set_bc(ctx, 0, 0, *r, K["farfield"], None, None) == -1
    assert lib.cfd_set_bc(ctx, 0, 0, *r, K["farfield"], arr(1.0, 0.5, 0.0, -0.7), None) == -6
    assert lib.cfd_set_bc(ctx, 0, 0, *r, K["farfield"], arr(1.0, float("nan"), 0.0, 0.7), None) == -6
    assert lib.cfd_set_bc(ctx, 0, 0, *r, K["sub_inflow"], arr(0.0, 1.0, 1.0, 0.0), None) == -6
    assert lib.cfd_set_bc(ctx, 0, 0, *r, K["sub_inflow"], arr(0.9, 1.1, 0.0, 0.0), None) == -1
    assert lib.cfd_set_bc(ctx, 0, 1, *r, K["sub_outflow"], arr(-0.7), None) == -6
    pid = ctypes.c_int()
    assert lib.cfd_set_bc(ctx, 0, 0, *r, K["sub_inflow"], arr(0.9, 1.1, 2.0, 0.0), ctypes.byref(pid)) == 0
    assert lib.cfd_set_bc(ctx, 0, 1, *r, K["sub_outflow"], arr(0.7), None) == 0
    assert lib.cfd_set_bc(ctx, 0, 2, *rj, K["slip_wall"], None, None) == 0
    assert lib.cfd_set_bc(ctx, 0, 3, *rj, K["farfield"], arr(1.0, 0.5, 0.0, 0.7), None) == 0
    assert lib.cfd_set_bc(ctx, 0, 3, *rj, 8, None, None) == -1
    n = ctypes.c_size_t()
    assert lib.cfd_finalize(ctx, ctypes.byref(n)) == 0
    lib.cfd_destroy(ctx)
    # the residual VJP rejects the characteristic boundaries
    ctx = _ctx(capi, lib)
    _add(capi, lib, ctx, 8, 6)
    assert lib.cfd_enable_adjoint(ctx, 1) == 0
    assert lib.cfd_set_bc(ctx, 0, 0, *r, K["farfield"], arr(1.0, 0.5, 0.0, 0.7), None) == 0
    assert lib.cfd_set_bc(ctx, 0, 1, *r, K["extrap_outflow"], None, None) == 0
    assert lib.cfd_connect(ctx, 0, 2, *rj, 0, 3, *rj, 0) == 0
    assert lib.cfd_finalize(ctx, ctypes.byref(n)) == -7
    assert b"residual VJP" in lib.cfd_last_error(ctx)
    lib.cfd_destroy(ctx)


def test_limiter_freezing_validation():
    capi, lib = _lib()
    ctx = _ctx(capi, lib, limiter=0)
    assert lib.cfd_enable_limiter_freezing(ctx, 1) == -1  # nothing to freeze
    lib.cfd_destroy(ctx)
    ctx = _ctx(capi, lib)
    _add(capi, lib, ctx, 8, 6)
    _periodic(capi, lib, ctx, 0, 8, 6)
    n0 = ctypes.c_size_t()
    assert lib.cfd_finalize(ctx, ctypes.byref(n0)) == 0
    assert lib.cfd_enable_limiter_freezing(ctx, 1) == -2  # after finalize
    assert lib.cfd_freeze_limiter(ctx, 1) == -2           # no workspace, not enabled
    lib.cfd_destroy(ctx)
    # the frozen factors take dim * nvar padded arrays of workspace
    ctx = _ctx(capi, lib)
    _add(capi, lib, ctx, 8, 6)
    _periodic(capi, lib, ctx, 0, 8, 6)
    assert lib.cfd_enable_limiter_freezing(ctx, 1) == 0
    n1 = ctypes.c_size_t()
    assert lib.cfd_finalize(ctx, ctypes.byref(n1)) == 0
    assert n1.value >= n0.value + 2 * 4 * (8 + 4) * (6 + 4) * 8
    lib.cfd_destroy(ctx)
    # not with the adjoint
    ctx = _ctx(capi, lib)
    _add(capi, lib, ctx, 8, 6)
    _periodic(capi, lib, ctx, 0, 8, 6)
    assert lib.cfd_enable_limiter_freezing(ctx, 1) == 0
    assert lib.cfd_enable_adjoint(ctx, 1) == 0
    assert lib.cfd_finalize(ctx, ctypes.byref(n1)) == -7
    lib.cfd_destroy(ctx)


def test_navier_stokes_config_validation():
    capi, lib = _lib()
    ctx = ctypes.c_void_p()
    assert lib.cfd_create(ctypes.byref(_cfg(capi, viscosity=-1e-3)), None, ctypes.byref(ctx)) == -1
    assert lib.cfd_create(ctypes.byref(_cfg(capi, viscosity=1e-3, prandtl=0.0)), None, ctypes.byref(ctx)) == -1
    # the viscous workspace: centres, pseudo-nodes, viscous residual
    n0, n1 = ctypes.c_size_t(), ctypes.c_size_t()
    for visc, n in ((0.0, n0), (1e-3, n1)):
        ctx = _ctx(capi, lib, viscosity=visc, prandtl=0.72)
        _add(capi, lib, ctx, 8, 6)
        _periodic(capi, lib, ctx, 0, 8, 6)
        assert lib.cfd_finalize(ctx, ctypes.byref(n)) == 0
        lib.cfd_destroy(ctx)
    assert n1.value >= n0.value + 8 * (9 * 7 * (2 + 3) + 48 * 3)
    # no-slip walls take no parameters; the adjoint rejects viscosity
    ctx = _ctx(capi, lib, viscosity=1e-3, prandtl=0.72)
    _add(capi, lib, ctx, 8, 6)
    r = (capi.int2([0]), capi.int2([8]))
    assert lib.cfd_set_bc(ctx, 0, 2, *r, capi.BC["noslip_wall"], None, None) == 0
    assert lib.cfd_set_bc(ctx, 0, 3, *r, capi.BC["noslip_wall"], None, None) == 0
    assert lib.cfd_connect(ctx, 0, 0, capi.int2([0]), capi.int2([6]), 0, 1, capi.int2([0]), capi.int2([6]), 0) == 0
    assert lib.cfd_enable_adjoint(ctx, 1) == 0
    n = ctypes.c_size_t()
    assert lib.cfd_finalize(ctx, ctypes.byref(n)) == -7
    assert b"Euler" in lib.cfd_last_error(ctx)
    lib.cfd_destroy(ctx)


def test_topology_errors():
    capi, lib = _lib()
    ctx = _ctx(capi, lib)
    _add(capi, lib, ctx, 8, 6)
    _add(capi, lib, ctx, 8, 5)
    # extents differ (6 vs 5)
    assert lib.cfd_connect(ctx, 0, 1, capi.int2([0]), capi.int2([6]), 1, 0, capi.int2([0]), capi.int2([5]), 0) == -3
    lib.cfd_destroy(ctx)
    # a face without boundary condition
    ctx = _ctx(capi, lib)
    _add(capi, lib, ctx, 8, 6)
    assert lib.cfd_connect(ctx, 0, 0, capi.int2([0]), capi.int2([6]), 0, 1, capi.int2([0]), capi.int2([6]), 0) == 0
    n = ctypes.c_size_t()
    assert lib.cfd_finalize(ctx, ctypes.byref(n)) == -3
    assert b"without a boundary condition" in lib.cfd_last_error(ctx)
    lib.cfd_destroy(ctx)
    # overlapping definitions on one face
    ctx = _ctx(capi, lib)
    _add(capi, lib, ctx, 8, 6)
    _periodic(capi, lib, ctx, 0, 8, 6)
    assert lib.cfd_set_bc(ctx, 0, 2, capi.int2([2]), capi.int2([5]), 3, None, None) == 0
    assert lib.cfd_finalize(ctx, ctypes.byref(n)) == -3
    assert b"overlapping" in lib.cfd_last_error(ctx)
    lib.cfd_destroy(ctx)


def test_calls_out_of_order():
    capi, lib = _lib()
    ctx = _ctx(capi, lib)
    _add(capi, lib, ctx, 8, 6)
    _periodic(capi, lib, ctx, 0, 8, 6)
    buf = ctypes.c_void_p(4096)
    assert lib.cfd_residual(ctx, buf) == -2          # not finalized
    n = ctypes.c_size_t()
    assert lib.cfd_finalize(ctx, ctypes.byref(n)) == 0
    assert lib.cfd_rk_step(ctx, 1, None) == -2        # no workspace
    assert _add(capi, lib, ctx, 8, 8)[0] == -2         # after finalize
    assert lib.cfd_enable_adjoint(ctx, 1) == -2       # after finalize
    # binding without a device reports a HIP error on this host
    assert lib.cfd_bind_workspace(ctx, ctypes.c_void_p(4096), n.value) == -5
    lib.cfd_destroy(ctx)


def test_tile_lists_cover_every_cell_once():
    """Planning view: the tile count per variant covers the block exactly."""
    capi, lib = _lib()
    ctx = _ctx(capi, lib, dim=3)
    st, _ = _add(capi, lib, ctx, 40, 36, 34, dim=3)
    assert st == 0
    for a, (n1, n2) in enumerate([(36, 34), (40, 34), (40, 36)]):
        assert lib.cfd_connect(ctx, 0, 2 * a, capi.int2([0, 0]), capi.int2([n1, n2]), 0, 2 * a + 1,
                               capi.int2([0, 0]), capi.int2([n1, n2]), 0) == 0
    n = ctypes.c_size_t()
    assert lib.cfd_finalize(ctx, ctypes.byref(n)) == 0
    v = ctypes.c_longlong()
    nvar = ctypes.c_longlong()
    lib.cfd_query(ctx, capi.Q["nvariants"], ctypes.byref(nvar))
    import math
    for var in range(nvar.value):
        assert lib.cfd_set_variant(ctx, var) == 0
        lib.cfd_query(ctx, capi.Q["tile_x"], ctypes.byref(v))
        tx = v.value
        lib.cfd_query(ctx, capi.Q["tile_y"], ctypes.byref(v))
        ty = v.value
        lib.cfd_query(ctx, capi.Q["ntiles"], ctypes.byref(v))
        assert v.value >= math.ceil(40 / tx) * math.ceil(36 / ty)
    lib.cfd_destroy(ctx)


def test_debug_flags_validation():
    capi, lib = _lib()
    ctx = ctypes.c_void_p()
    assert lib.cfd_create(ctypes.byref(_cfg(capi, debug_flags=4)), None, ctypes.byref(ctx)) == -1
    assert lib.cfd_create(ctypes.byref(_cfg(capi, debug_flags=-1)), None, ctypes.byref(ctx)) == -1
    for flags in (0, capi.CHECK_FINITE, capi.NAN_GHOSTS, capi.CHECK_FINITE | capi.NAN_GHOSTS):
        ctx = _ctx(capi, lib, debug_flags=flags)
        _add(capi, lib, ctx, 8, 6)
        _periodic(capi, lib, ctx, 0, 8, 6)
        n = ctypes.c_size_t()
        assert lib.cfd_finalize(ctx, ctypes.byref(n)) == 0
        lib.cfd_destroy(ctx)


def test_config_struct_layout_matches_header(tmp_path):
    """The ctypes mirror of cfd_config has the C struct's size and field
    offsets (compiled from the header with the host C compiler)."""
    import shutil
    import subprocess
    from paper_2012_02925_amd import capi

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    fields = [f for f, _ in capi.CfdConfig._fields_]
    src = tmp_path / "layout.c"
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "cfdhip.h"', "int main(void) {",
             '  printf("%zu\\n", sizeof(cfd_config));']
    for f in fields:
        lines.append('  printf("%%zu\\n", offsetof(cfd_config, %s));' % f)
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert out[0] == ctypes.sizeof(capi.CfdConfig)
    for f, off in zip(fields, out[1:]):
        assert getattr(capi.CfdConfig, f).offset == off, f
