"""The C-ABI library loads, exports every symbol include/proxskip.h declares, and rejects bad
arguments on the host before any device work (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    text = open(os.path.join(ROOT, "include", "proxskip.h")).read()
    return re.findall(r"^PS_API\s+[\w\s\*]+?\b(\w+)\(", text, flags=re.M)


@pytest.fixture(scope="module")
def nat():
    from paper_2602_09527_amd import _native
    _native.load()
    return _native


def test_exports_every_declared_symbol(nat):
    declared = _header_symbols()
    assert len(declared) >= 20
    assert set(declared) == set(nat.EXPORTS)
    lib = C.CDLL(nat.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


def _desc(nat, **kw):
    d = dict(nx=16, ny=16, nz=1, n_angles=12, angles=None, n_bins=20, bin_width=1.0,
             det_offset=0.0, n_subsets=3, dtype=nat.PS_F32)
    d.update(kw)
    return nat.GeometryDesc(**d)


@pytest.mark.parametrize("bad", [dict(nx=0), dict(ny=-1), dict(nz=0), dict(n_angles=0),
                                 dict(n_bins=0), dict(bin_width=0.0), dict(bin_width=float("nan")),
                                 dict(n_subsets=0), dict(n_subsets=13), dict(dtype=7),
                                 dict(det_offset=float("inf"))])
def test_make_geometry_rejects(nat, bad):
    lib = nat.load()
    h = C.c_void_p()
    st = lib.make_geometry(C.byref(_desc(nat, **bad)), C.byref(h))
    assert st == nat.PS_EINVAL
    assert lib.last_error_message()


def test_make_geometry_unsupported(nat):
    lib = nat.load()
    h = C.c_void_p()
    assert lib.make_geometry(C.byref(_desc(nat, nx=5000)), C.byref(h)) == nat.PS_EUNSUPPORTED
    assert lib.make_geometry(C.byref(_desc(nat, n_bins=4096)), C.byref(h)) == nat.PS_EUNSUPPORTED


def test_geometry_queries_and_not_uploaded(nat):
    lib = nat.load()
    h = C.c_void_p()
    assert lib.make_geometry(C.byref(_desc(nat, n_angles=14, n_subsets=4)), C.byref(h)) == nat.PS_OK
    try:
        assert [lib.subset_size(h, i) for i in range(4)] == [4, 4, 3, 3]
        assert lib.subset_size(h, -1) == 14 and lib.subset_size(h, 4) == -1
        assert lib.geometry_device_bytes(h) > 0
        assert lib.tv_prox_workspace_bytes(h) > 0
        # upload needs a 256-byte aligned device buffer of the right size
        assert lib.geometry_upload(h, None, 1 << 20, None) == nat.PS_EINVAL
        assert lib.geometry_upload(h, C.c_void_p(256), 1, None) == nat.PS_EINVAL
        # nothing is queued before the tables are uploaded
        assert lib.project_subset(h, 0, C.c_void_p(256), C.c_void_p(256), None, 0, None) == nat.PS_EINVAL
        assert lib.backproject_subset(h, 0, C.c_void_p(256), C.c_void_p(256), 0, None, 0, None) == nat.PS_EINVAL
        assert lib.project_subset(h, 9, C.c_void_p(256), C.c_void_p(256), None, 0, None) == nat.PS_EINVAL
        # tv prox argument checks
        assert lib.tv_prox_fgp(h, C.c_void_p(256), C.c_void_p(256), -1.0, 5, 1, None, None, 0, None) == nat.PS_EINVAL
        assert lib.tv_prox_fgp(h, C.c_void_p(256), C.c_void_p(256), 0.1, -5, 1, None, None, 0, None) == nat.PS_EINVAL
        assert lib.tv_prox_fgp(h, C.c_void_p(256), C.c_void_p(256), 0.1, 5, 2, None, None, 0, None) == nat.PS_EINVAL
        assert lib.tv_prox_fgp(h, C.c_void_p(2), C.c_void_p(256), 0.1, 5, 1, None, None, 0, None) == nat.PS_EINVAL
    finally:
        lib.free_geometry(h)


@pytest.mark.parametrize("bad", [dict(gamma=0.0), dict(gamma=float("inf")), dict(p=0.0), dict(p=1.5),
                                 dict(alpha=-1.0), dict(fgp_inner=-1), dict(nonneg=2),
                                 dict(n_epochs=-1), dict(plain_prox_svrg=3), dict(k0=1),
                                 dict(k0=-3), dict(tol_rel_change=-1.0), dict(estimator=3),
                                 dict(estimator=-1)])
def test_solver_params_rejected(nat, bad):
    lib = nat.load()
    h = C.c_void_p()
    assert lib.make_geometry(C.byref(_desc(nat)), C.byref(h)) == nat.PS_OK
    try:
        prm = dict(gamma=1e-3, p=0.5, alpha=0.1, fgp_inner=5, nonneg=1, n_epochs=2,
                   plain_prox_svrg=0, seed=1, k0=0, tol_rel_change=0.0)
        prm.update(bad)
        P = nat.SolverParams(**prm)
        s = C.c_void_p()
        fake = C.c_void_p(256)
        st = lib.solver_init(h, fake, fake, fake, fake, C.byref(P), fake, 1 << 30, C.byref(s))
        assert st == nat.PS_EINVAL
        assert not s.value
    finally:
        lib.free_geometry(h)


def test_sequences_match_oracle_bitwise(nat, orc):
    from paper_2602_09527_amd import api
    for seed, k0, count, N, p in [(0, 0, 1_000_000, 20, 0.1), (2**63 + 12345, 400, 100_000, 7, 0.02),
                                  (101, 0, 300, 10, 0.1), (5, 30, 1000, 1, 1.0), (9, 0, 5000, 30, 0.05)]:
        s1, c1 = api.sample_sequences(seed, k0, count, N, p)
        s2, c2 = orc.sequences(seed, k0, count, N, p)
        assert np.array_equal(s1, s2) and np.array_equal(c1, c2)


def test_refresh_coins_match_oracle_bitwise(nat, orc):
    from paper_2602_09527_amd import api
    for seed, k0, count, N in [(0, 0, 1_000_000, 20), (2**63 + 12345, 400, 100_000, 7),
                               (101, 0, 300, 10), (5, 30, 1000, 1), (9, 0, 5000, 30)]:
        assert np.array_equal(api.sample_refresh_coins(seed, k0, count, N),
                              orc.refresh_coins(seed, k0, count, N))
    lib = nat.load()
    assert lib.sample_refresh_coins(0, 0, 10, 0, None) == nat.PS_EINVAL
    assert lib.sample_refresh_coins(0, -1, 10, 4, None) == nat.PS_EINVAL


def test_sequences_reject(nat):
    lib = nat.load()
    assert lib.sample_sequences(0, 0, 10, 0, 0.5, None, None) == nat.PS_EINVAL
    assert lib.sample_sequences(0, 0, 10, 4, 0.0, None, None) == nat.PS_EINVAL
    assert lib.sample_sequences(0, -1, 10, 4, 0.5, None, None) == nat.PS_EINVAL


def test_plan_get_set_and_validation(nat):
    lib = nat.load()
    h = C.c_void_p()
    assert lib.make_geometry(C.byref(_desc(nat, nx=64, ny=64, n_angles=60, n_bins=96, n_subsets=6)),
                             C.byref(h)) == nat.PS_OK
    try:
        auto = nat.Plan()
        assert lib.geometry_get_plan(h, C.byref(auto)) == nat.PS_OK
        assert auto.proj_split_full >= 1 and auto.proj_split_subset >= 1
        assert 1 <= auto.bp_groups_full <= 16 and auto.bp_strip_full in (1, 2, 4, 8)
        assert auto.fgp_iters == 8 and (auto.fgp_waves, auto.fgp_rows) == (8, 4)
        # the scatter backprojector unless a plan asks for the gather
        assert (auto.bp_method_full, auto.bp_method_subset) == (1, 1)
        forced = nat.Plan(proj_split_full=2, proj_split_subset=1, bp_groups_full=4,
                          bp_groups_subset=2, bp_strip_full=4, bp_strip_subset=2, fgp_iters=5)
        assert lib.geometry_set_plan(h, C.byref(forced)) == nat.PS_OK
        got = nat.Plan()
        assert lib.geometry_get_plan(h, C.byref(got)) == nat.PS_OK
        assert (got.proj_split_full, got.proj_split_subset, got.bp_groups_full,
                got.bp_groups_subset, got.bp_strip_full, got.bp_strip_subset, got.fgp_iters) == \
            (2, 1, 4, 2, 4, 2, 5)
        for bad in (dict(proj_split_full=-1), dict(bp_groups_subset=17), dict(bp_strip_full=3),
                    dict(fgp_iters=17), dict(bp_method_subset=3), dict(fgp_waves=4, fgp_rows=2),
                    dict(fgp_waves=8), dict(fgp_rows=4), dict(fgp_waves=32, fgp_rows=2),
                    dict(fgp3d_form=6), dict(fgp3d_form=-1), dict(fgp3d_chunk=257),
                    dict(bp_gather_split=3), dict(fgp_cols=3), dict(fgp_cols=-1),
                    dict(bp_gather_fused=3), dict(bp_gather_fused=-1)):
            assert lib.geometry_set_plan(h, C.byref(nat.Plan(**bad))) == nat.PS_EINVAL
        # a rejected plan leaves the previous one in place
        assert lib.geometry_get_plan(h, C.byref(got)) == nat.PS_OK and got.fgp_iters == 5
        # a 2D FGP tile caps the inner iterations per launch at its height / 2 - 2
        for w, r, t, want in ((4, 4, 8, 6), (8, 2, 3, 3), (16, 4, 0, 8), (4, 8, 7, 7), (16, 4, 16, 16),
                              (8, 8, 12, 12), (16, 2, 16, 14)):
            assert lib.geometry_set_plan(h, C.byref(nat.Plan(fgp_waves=w, fgp_rows=r, fgp_iters=t))) == nat.PS_OK
            assert lib.geometry_get_plan(h, C.byref(got)) == nat.PS_OK
            assert (got.fgp_waves, got.fgp_rows, got.fgp_iters) == (w, r, want)
        # workspace sizes follow the plan
        zero = nat.Plan()
        assert lib.geometry_set_plan(h, C.byref(zero)) == nat.PS_OK
        ws_auto = lib.backproject_workspace_bytes(h, -1)
        assert lib.geometry_set_plan(h, C.byref(nat.Plan(bp_groups_full=1))) == nat.PS_OK
        assert lib.backproject_workspace_bytes(h, -1) <= ws_auto
        assert lib.geometry_autotune_workspace_bytes(h) > 0
        # autotuning needs uploaded tables: refused on the host
        assert lib.geometry_autotune(h, None, 0, 3, None, None) == nat.PS_EINVAL
    finally:
        lib.free_geometry(h)


@pytest.mark.parametrize("bad", [dict(gamma=0.0), dict(gamma=float("nan")), dict(alpha=-1.0),
                                 dict(fgp_inner=-1), dict(nonneg=2), dict(n_iters=-1), dict(t=0.5),
                                 dict(t=None)])
def test_fista_arguments_rejected(nat, bad):
    lib = nat.load()
    h = C.c_void_p()
    assert lib.make_geometry(C.byref(_desc(nat)), C.byref(h)) == nat.PS_OK
    try:
        assert lib.fista_workspace_bytes(h) > 0 and lib.fista_workspace_bytes(None) == 0
        a = dict(gamma=1e-3, alpha=0.1, fgp_inner=5, nonneg=1, n_iters=3, t=1.0)
        a.update(bad)
        t = None if a["t"] is None else C.byref(C.c_double(a["t"]))
        fake = C.c_void_p(256)
        st = lib.fista_run(h, fake, fake, fake, fake, t, a["gamma"], a["alpha"], a["fgp_inner"],
                           a["nonneg"], a["n_iters"], fake, 1 << 30, None)
        assert st == nat.PS_EINVAL
    finally:
        lib.free_geometry(h)


@pytest.mark.parametrize("bad", [dict(alpha=-1.0), dict(alpha=float("inf")), dict(nonneg=3),
                                 dict(n_iters=-2)])
def test_pdhg_arguments_rejected(nat, bad):
    lib = nat.load()
    h = C.c_void_p()
    assert lib.make_geometry(C.byref(_desc(nat)), C.byref(h)) == nat.PS_OK
    try:
        assert lib.pdhg_workspace_bytes(h) > 0 and lib.pdhg_workspace_bytes(None) == 0
        a = dict(alpha=0.1, nonneg=1, n_iters=3)
        a.update(bad)
        fake = C.c_void_p(256)
        st = lib.pdhg_run(h, fake, fake, fake, fake, a["alpha"], a["nonneg"], a["n_iters"], fake,
                          1 << 30, None)
        assert st == nat.PS_EINVAL
        assert b"alpha" in lib.last_error_message() or b"nonneg" in lib.last_error_message() \
            or b"n_iters" in lib.last_error_message()
    finally:
        lib.free_geometry(h)


def test_plan_fgp_tile_defaults_per_dtype(nat):
    lib = nat.load()
    for dt, tile in ((nat.PS_F32, (8, 4)), (nat.PS_F64, (16, 2))):
        h = C.c_void_p()
        assert lib.make_geometry(C.byref(_desc(nat, dtype=dt)), C.byref(h)) == nat.PS_OK
        try:
            got = nat.Plan()
            assert lib.geometry_get_plan(h, C.byref(got)) == nat.PS_OK
            assert (got.fgp_waves, got.fgp_rows, got.fgp_iters) == (*tile, 8)
            # deeper launches: up to 16 inner iterations in FP32, 8 in FP64
            deep = nat.Plan(fgp_waves=16, fgp_rows=4, fgp_iters=12)
            want = nat.PS_OK if dt == nat.PS_F32 else nat.PS_EINVAL
            assert lib.geometry_set_plan(h, C.byref(deep)) == want
        finally:
            lib.free_geometry(h)


def test_binding_structs_match_the_c_layout(nat, tmp_path):
    # the ctypes structures of the binding against the header as a C compiler lays it out
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    structs = {"ps_geometry_desc": nat.GeometryDesc, "ps_plan": nat.Plan,
               "ps_solver_params": nat.SolverParams, "ps_solver_stats": nat.SolverStats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "proxskip.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_noalloc_entry_rejects_on_the_host(nat):
    # proxskip_svrg_run_noalloc: parameter checks, a tolerance run, and a problem whose solver
    # scratch exceeds the static array are refused before any device call
    lib = nat.load()
    assert lib.proxskip_noalloc_max_bytes() == 64 << 20
    fake = C.c_void_p(256)
    good = dict(gamma=1e-3, p=0.5, alpha=0.1, fgp_inner=5, nonneg=1, n_epochs=2,
                plain_prox_svrg=0, seed=1, k0=0, tol_rel_change=0.0)
    h = C.c_void_p()
    assert lib.make_geometry(C.byref(_desc(nat)), C.byref(h)) == nat.PS_OK
    try:
        for bad in (dict(gamma=0.0), dict(p=1.5), dict(n_epochs=-1), dict(tol_rel_change=1e-4)):
            P = nat.SolverParams(**{**good, **bad})
            assert lib.proxskip_svrg_run_noalloc(h, fake, fake, fake, fake, C.byref(P), None,
                                                 None) == nat.PS_EINVAL
        assert lib.proxskip_svrg_run_noalloc(None, fake, fake, fake, fake,
                                             C.byref(nat.SolverParams(**good)), None, None) == nat.PS_EINVAL
    finally:
        lib.free_geometry(h)
    big = C.c_void_p()
    assert lib.make_geometry(C.byref(_desc(nat, nx=1024, ny=1024, n_angles=1800, n_bins=1448,
                                           n_subsets=30)), C.byref(big)) == nat.PS_OK
    try:
        P = nat.SolverParams(**good)
        assert lib.proxskip_workspace_bytes(big, C.byref(P)) > lib.proxskip_noalloc_max_bytes()
        assert lib.proxskip_svrg_run_noalloc(big, fake, fake, fake, fake, C.byref(P), None,
                                             None) == nat.PS_EINVAL
        assert b"static scratch" in lib.last_error_message()
    finally:
        lib.free_geometry(big)


def test_kernel_timer_arguments(nat):
    # measurement support: class masks and class numbers outside 1..9 are refused on the host
    lib = nat.load()
    ms, n = C.c_double(), C.c_int32()
    assert lib.kernel_timer_start(1) == nat.PS_EINVAL          # bit 0 is no class
    assert lib.kernel_timer_start(1 << 10) == nat.PS_EINVAL
    assert lib.kernel_timer_read(0, C.byref(ms), C.byref(n)) == nat.PS_EINVAL
    assert lib.kernel_timer_read(10, C.byref(ms), C.byref(n)) == nat.PS_EINVAL
    assert lib.kernel_timer_start((1 << 1) | (1 << 9)) == nat.PS_OK
    assert lib.kernel_timer_read(1, C.byref(ms), C.byref(n)) == nat.PS_OK
    assert n.value == 0 and ms.value == 0.0                    # nothing launched
    assert lib.kernel_timer_read(1, None, C.byref(n)) == nat.PS_EINVAL
    assert lib.kernel_timer_stop() == nat.PS_OK


def test_kernel_time_arguments(nat):
    lib = nat.load()
    h = C.c_void_p()
    assert lib.make_geometry(C.byref(_desc(nat)), C.byref(h)) == nat.PS_OK
    try:
        assert lib.kernel_time_workspace_bytes(h) > 0
        us = C.c_double()
        # not uploaded: refused before any device work
        assert lib.kernel_time(h, 1, 10, C.c_void_p(256), 1 << 30, None, C.byref(us)) == nat.PS_EINVAL
        assert lib.kernel_time(None, 1, 10, C.c_void_p(256), 1 << 30, None, C.byref(us)) == nat.PS_EINVAL
    finally:
        lib.free_geometry(h)


def test_device_alloc_arguments(nat):
    lib = nat.load()
    p, contig = C.c_void_p(), C.c_int32(7)
    # refused on the host before any HIP call
    assert lib.device_alloc(0, 0, C.byref(p), C.byref(contig)) == nat.PS_EINVAL
    assert p.value is None and contig.value == 0
    assert lib.device_alloc(1 << 20, 0, None, None) == nat.PS_EINVAL
    assert lib.device_free(None) == nat.PS_OK


@pytest.mark.parametrize("dtype,form", [(0, 5), (1, 2)], ids=["f32", "f64"])
def test_automatic_3d_form_per_dtype(nat, dtype, form):
    # two inner iterations per launch: 8 x 4 wave tiles in FP32, 8 x 2 in FP64 (whose 8 x 4 tile
    # needs all 256 registers); chunks of 16 slices
    lib = nat.load()
    h = C.c_void_p()
    d = _desc(nat, nx=40, ny=30, nz=5, n_angles=12, n_bins=50, n_subsets=3, dtype=dtype)
    assert lib.make_geometry(C.byref(d), C.byref(h)) == nat.PS_OK
    try:
        got = nat.Plan()
        assert lib.geometry_get_plan(h, C.byref(got)) == nat.PS_OK
        assert (got.fgp3d_form, got.fgp3d_chunk) == (form, 16)
        assert lib.geometry_set_plan(h, C.byref(nat.Plan(fgp3d_form=1))) == nat.PS_OK
        assert lib.geometry_get_plan(h, C.byref(got)) == nat.PS_OK
        assert (got.fgp3d_form, got.fgp3d_chunk) == (1, 4)
    finally:
        lib.free_geometry(h)


def test_gather_fused_plan_rule(nat):
    # the subset gather adds the projector's partials itself only where both apply: the gather
    # backprojects subsets and the projector splits rays; automatic up to 8 partials per ray
    lib = nat.load()
    got = nat.Plan()

    def fused(h, **plan):
        assert lib.geometry_set_plan(h, C.byref(nat.Plan(**plan))) == nat.PS_OK
        assert lib.geometry_get_plan(h, C.byref(got)) == nat.PS_OK
        return got.bp_gather_fused, got.proj_split_subset

    for ext, split in ((128, 4), (512, 16)):
        h = C.c_void_p()
        d = _desc(nat, nx=ext, ny=ext, n_angles=12, n_bins=ext + ext // 2, n_subsets=3)
        assert lib.make_geometry(C.byref(d), C.byref(h)) == nat.PS_OK
        try:
            assert fused(h) == (1, split)                                   # scatter
            assert fused(h, bp_method_subset=2) == (2 if split <= 8 else 1, split)
            assert fused(h, bp_method_subset=2, proj_split_subset=4) == (2, 4)
            assert fused(h, bp_method_subset=2, proj_split_subset=1) == (1, 1)
            assert fused(h, bp_method_subset=2, bp_gather_fused=1) == (1, split)
            assert fused(h, bp_method_subset=2, bp_gather_fused=2) == (2, split)
            assert fused(h, bp_method_subset=1, bp_gather_fused=2) == (1, split)
        finally:
            lib.free_geometry(h)
    # automatic only while the partials take at most 32 MiB: 4 x 256 slices x 20 angles x 768
    # bins x 4 bytes = 63 MB is not fused unless the plan asks for it
    h = C.c_void_p()
    d = _desc(nat, nx=512, ny=512, nz=256, n_angles=60, n_bins=768, n_subsets=3)
    assert lib.make_geometry(C.byref(d), C.byref(h)) == nat.PS_OK
    try:
        assert fused(h, bp_method_subset=2, proj_split_subset=4) == (1, 4)
        assert fused(h, bp_method_subset=2, proj_split_subset=4, bp_gather_fused=2) == (2, 4)
        assert lib.geometry_set_plan(h, C.byref(nat.Plan(bp_method_subset=2, proj_split_subset=4))) == nat.PS_OK
        assert lib.project_workspace_bytes(h, 0) == 4 * 256 * 20 * 768 * 4
    finally:
        lib.free_geometry(h)
    # no gather when bins are closer than a pixel, so never fused
    h = C.c_void_p()
    d = _desc(nat, nx=128, ny=128, n_angles=12, n_bins=400, bin_width=0.5, n_subsets=3)
    assert lib.make_geometry(C.byref(d), C.byref(h)) == nat.PS_OK
    try:
        assert fused(h, bp_method_subset=2, bp_gather_fused=2) == (1, 4)
    finally:
        lib.free_geometry(h)
