"""The C ABI without a GPU: the library loads, exports every call include/mvgs.h declares, and
rejects invalid arguments with MVGS_EINVAL before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2506_12727_amd import _lib as L
from paper_2506_12727_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mvgs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mvgs_\w+)\s*\(", src)))


def test_header_declarations_are_exported():
    lib = L.lib()
    names = _declared()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTED)


def test_status_strings():
    lib = L.lib()
    for code in (L.MVGS_OK, L.MVGS_EINVAL, L.MVGS_ENOMEM, L.MVGS_ECAPACITY, L.MVGS_EHIP, L.MVGS_ERETRY):
        assert lib.mvgs_status_string(code)
    assert lib.mvgs_status_string(-99) == b"unknown status"


@pytest.fixture()
def ctx():
    lib = L.lib()
    h = C.c_void_p()
    assert lib.mvgs_create(C.byref(h), None) == L.MVGS_OK
    yield h
    lib.mvgs_destroy(h)


def test_create_rejects_bad_tiles():
    lib = L.lib()
    for tw, th, ppl in [(4, 16, 0), (16, 12, 0), (64, 16, 0), (-8, 8, 0), (16, 16, 3), (8, 16, 4), (16, 8, 2), (16, 8, 4)]:
        o = L.mvgs_options()
        o.tile_w, o.tile_h, o.pixels_per_lane = tw, th, ppl
        h = C.c_void_p()
        assert lib.mvgs_create(C.byref(h), C.byref(o)) == L.MVGS_EINVAL
    for tw, th, ppl in [(16, 16, 0), (16, 16, 1), (16, 32, 4), (8, 8, 1), (32, 16, 2), (16, 16, 4)]:
        o = L.mvgs_options()
        o.tile_w, o.tile_h, o.pixels_per_lane = tw, th, ppl
        h = C.c_void_p()
        assert lib.mvgs_create(C.byref(h), C.byref(o)) == L.MVGS_OK
        lib.mvgs_destroy(h)
    assert lib.mvgs_create(None, None) == L.MVGS_EINVAL


def _gauss(P=10, deg=0, ptr=0x1000):
    g = L.mvgs_gaussians()
    g.P, g.sh_degree = P, deg
    g.means = g.scales = g.quats = g.opacities = g.sh = ptr
    return g


def _fwd(ctx, g, cams, images="auto"):
    lib = L.lib()
    ca = L.camera_array(cams) if cams is not None else None
    n = len(cams) if cams is not None else 0
    if images == "auto":
        images = L.ptr_array([0x2000] * max(n, 1))
    fr = C.c_void_p()
    return lib.mvgs_forward(ctx, None, C.byref(g) if g is not None else None, ca, n, images, C.byref(fr))


def _err(ctx):
    return L.lib().mvgs_last_error(ctx).decode()


def test_forward_argument_validation(ctx):
    cams = scenes.make_cameras([(64, 48), (32, 32)])
    assert _fwd(ctx, None, cams) == L.MVGS_EINVAL
    assert _fwd(ctx, _gauss(deg=4), cams) == L.MVGS_EINVAL and "sh_degree" in _err(ctx)
    assert _fwd(ctx, _gauss(P=-1), cams) == L.MVGS_EINVAL
    assert _fwd(ctx, _gauss(P=5, ptr=0), cams) == L.MVGS_EINVAL and "NULL" in _err(ctx)
    assert _fwd(ctx, _gauss(), []) == L.MVGS_EINVAL                       # B = 0
    assert _fwd(ctx, _gauss(), cams, images=None) == L.MVGS_EINVAL
    assert _fwd(ctx, _gauss(), cams, images=L.ptr_array([0x2000, 0])) == L.MVGS_EINVAL
    bad = scenes.make_cameras([(64, 48)])
    bad[0].fx = 0.0
    assert _fwd(ctx, _gauss(), bad) == L.MVGS_EINVAL and "focal" in _err(ctx)
    bad = scenes.make_cameras([(0, 48)])
    assert _fwd(ctx, _gauss(), bad) == L.MVGS_EINVAL
    # 4096 x 4096 at 16x16 is exactly 65536 tiles (allowed); one more column of tiles is not
    big = scenes.make_cameras([(4097, 4096)])
    assert _fwd(ctx, _gauss(), big) == L.MVGS_EINVAL and "tiles" in _err(ctx)
    lib = L.lib()
    assert lib.mvgs_forward(ctx, None, C.byref(_gauss()), L.camera_array(cams), 2,
                            L.ptr_array([0x2000] * 2), None) == L.MVGS_EINVAL
    assert lib.mvgs_forward(None, None, None, None, 0, None, None) == L.MVGS_EINVAL


def test_loss_and_backward_validation(ctx):
    lib = L.lib()
    cams = scenes.make_cameras([(16, 16)])
    ca = L.camera_array(cams)
    p = L.ptr_array([0x2000])
    assert lib.mvgs_loss(ctx, None, ca, 0, p, p, 1.0, 0.0, 0x3000, p) == L.MVGS_EINVAL
    assert lib.mvgs_loss(ctx, None, ca, 1, None, p, 1.0, 0.0, 0x3000, p) == L.MVGS_EINVAL
    assert lib.mvgs_loss(ctx, None, ca, 1, p, p, float("nan"), 0.0, 0x3000, p) == L.MVGS_EINVAL
    # the no-alloc variant validates alike and refuses, before any device work, what its fixed
    # scratch cannot hold: more than 64 views, or the partial sums of D-SSIM over ~1.4G pixels
    assert lib.mvgs_loss_noalloc(ctx, None, ca, 0, p, p, 1.0, 0.0, 0x3000, p) == L.MVGS_EINVAL
    assert lib.mvgs_loss_noalloc(ctx, None, ca, 1, None, p, 1.0, 0.0, 0x3000, p) == L.MVGS_EINVAL
    assert lib.mvgs_loss_noalloc(ctx, None, ca, 1, p, p, 1.0, 0.0, None, p) == L.MVGS_EINVAL
    many = scenes.make_cameras([(16, 16)] * 65)
    p65 = L.ptr_array([0x2000] * 65)
    assert lib.mvgs_loss_noalloc(ctx, None, L.camera_array(many), 65, p65, p65, 1.0, 0.0, 0x3000,
                                 p65) == L.MVGS_ECAPACITY
    # 24 views of 8192x8192 (65,536 tiles each at 32x32): 1.6G pixels, D-SSIM partials 37.7 MB
    o = L.mvgs_options()
    o.tile_w = o.tile_h = 32
    c32 = C.c_void_p()
    assert lib.mvgs_create(C.byref(c32), C.byref(o)) == L.MVGS_OK
    huge = scenes.make_cameras([(8192, 8192)] * 24)
    p24 = L.ptr_array([0x2000] * 24)
    assert lib.mvgs_loss_noalloc(c32, None, L.camera_array(huge), 24, p24, p24, 0.8, 0.2, 0x3000,
                                 p24) == L.MVGS_ECAPACITY
    assert "scratch" in _err(c32)
    lib.mvgs_destroy(c32)
    gr = L.mvgs_grads()
    assert lib.mvgs_backward(ctx, None, C.byref(_gauss()), None, p, C.byref(gr), None) == L.MVGS_EINVAL
    assert lib.mvgs_frame_release(ctx, None) == L.MVGS_EINVAL
    assert lib.mvgs_frame_info(None, None, None, None) == L.MVGS_EINVAL
    assert lib.mvgs_export_binning(ctx, None, None, None, None, None) == L.MVGS_EINVAL


def test_product_path_has_no_oracle_dependency():
    """The GPU package never imports the oracle (the oracle is test infrastructure)."""
    pkg = os.path.join(ROOT, "paper_2506_12727_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src and "liboracle" not in src, f


def test_workspace_limit_options_and_memory_queries():
    lib = L.lib()
    o = L.mvgs_options()
    o.workspace_limit = -1
    h = C.c_void_p()
    assert lib.mvgs_create(C.byref(h), C.byref(o)) == L.MVGS_EINVAL
    o = L.mvgs_options()
    o.reserved0 = 5
    assert lib.mvgs_create(C.byref(h), C.byref(o)) == L.MVGS_EINVAL
    # capacities: both or neither, non-negative, below 2^32
    for cv, ck in [(10, 0), (0, 10), (-1, -1), (1 << 32, 10), (10, 1 << 32)]:
        o = L.mvgs_options()
        o.capacity_records, o.capacity_pairs = cv, ck
        assert lib.mvgs_create(C.byref(h), C.byref(o)) == L.MVGS_EINVAL, (cv, ck)
    o = L.mvgs_options()
    o.capacity_records, o.capacity_pairs = 1000, 5000
    assert lib.mvgs_create(C.byref(h), C.byref(o)) == L.MVGS_OK
    assert lib.mvgs_frame_check(h, None, None) == L.MVGS_EINVAL
    assert lib.mvgs_frame_check(None, None, None) == L.MVGS_EINVAL
    assert lib.mvgs_frame_set_cameras(h, None, None, 1) == L.MVGS_EINVAL
    lib.mvgs_destroy(h)
    o = L.mvgs_options()
    o.workspace_limit = 1 << 30
    assert lib.mvgs_create(C.byref(h), C.byref(o)) == L.MVGS_OK
    held = C.c_int64(-1)
    # a fresh context holds no device memory; the query makes no HIP call
    assert lib.mvgs_memory_held(h, C.byref(held)) == L.MVGS_OK and held.value == 0
    assert lib.mvgs_memory_held(h, None) == L.MVGS_EINVAL
    assert lib.mvgs_set_workspace_limit(h, -5) == L.MVGS_EINVAL
    assert lib.mvgs_set_workspace_limit(h, 0) == L.MVGS_OK
    assert lib.mvgs_set_workspace_limit(None, 0) == L.MVGS_EINVAL
    assert lib.mvgs_frame_workspace(None, C.byref(held)) == L.MVGS_EINVAL
    lib.mvgs_destroy(h)


def test_partial_and_subsample_validation(ctx):
    lib = L.lib()
    g = _gauss()
    cams = scenes.make_cameras([(32, 32), (32, 32)])
    ca = L.camera_array(cams)
    imgs = L.ptr_array([0x2000, 0x2000])
    fr = C.c_void_p()

    def part(off, pix, n, mode):
        return lib.mvgs_forward_partial(ctx, None, C.byref(g), ca, 2, off, pix, n, mode, imgs, C.byref(fr))

    assert part(0x3000, 0x4000, 10, 7) == L.MVGS_EINVAL
    assert "mode" in _err(ctx)
    assert part(0x3000, 0x4000, -1, 0) == L.MVGS_EINVAL
    assert part(0x3000, 0x4000, 1 << 32, 0) == L.MVGS_EINVAL
    assert part(None, 0x4000, 10, 0) == L.MVGS_EINVAL
    assert part(0x3000, None, 10, 1) == L.MVGS_EINVAL
    assert "NULL" in _err(ctx)
    # camera validation applies as in the full forward
    bad = L.camera_array(scenes.make_cameras([(0, 32)]))
    assert lib.mvgs_forward_partial(ctx, None, C.byref(g), bad, 1, 0x3000, 0x4000, 1, 0, imgs,
                                    C.byref(fr)) == L.MVGS_EINVAL
    # sub-sampling needs views of one size and non-NULL buffers
    mixed = L.camera_array(scenes.make_cameras([(32, 32), (33, 32)]))
    assert lib.mvgs_subsample(ctx, None, mixed, 2, 0x1000, 0x2000, 0x3000) == L.MVGS_EINVAL
    assert "one size" in _err(ctx)
    assert lib.mvgs_subsample(ctx, None, ca, 2, None, 0x2000, 0x3000) == L.MVGS_EINVAL
    assert lib.mvgs_subsample(ctx, None, ca, 0, 0x1000, 0x2000, 0x3000) == L.MVGS_EINVAL


def test_adapt_density_validation(ctx):
    lib = L.lib()
    g = _gauss()
    prm = L.mvgs_adc_params(2e-4, 2e-4, 0.01, 0.005)
    out = L.mvgs_gaussians_out(0x5000, 0x5000, 0x5000, 0x5000, 0x5000)
    n = C.c_int64(-7)

    def call(g=g, e1=0x1000, normals=0x4000, prm=prm, out=out, cap=20, n=n):
        return lib.mvgs_adapt_density(ctx, None, C.byref(g) if g is not None else None, e1, 0x2000, 0x3000, normals,
                                      C.byref(prm) if prm is not None else None,
                                      C.byref(out) if out is not None else None, 0x6000, cap,
                                      C.byref(n) if n is not None else None)

    assert call(g=None) == L.MVGS_EINVAL
    assert call(g=_gauss(deg=4)) == L.MVGS_EINVAL
    assert call(e1=None) == L.MVGS_EINVAL and "NULL" in _err(ctx)
    assert call(normals=None) == L.MVGS_EINVAL
    assert call(prm=None) == L.MVGS_EINVAL
    assert call(out=None) == L.MVGS_EINVAL
    assert call(n=None) == L.MVGS_EINVAL
    assert call(cap=-1) == L.MVGS_EINVAL and "capacity" in _err(ctx)
    assert call(prm=L.mvgs_adc_params(float("nan"), 2e-4, 0.01, 0.005)) == L.MVGS_EINVAL
    assert call(prm=L.mvgs_adc_params(2e-4, 2e-4, -1.0, 0.005)) == L.MVGS_EINVAL and "finite" in _err(ctx)
    assert lib.mvgs_adapt_density(None, None, None, None, None, None, None, None, None, None, 0, None) == L.MVGS_EINVAL


def test_create_rejects_half_an_allocator():
    lib = L.lib()
    keep = L.ALLOC_FN(lambda n, c: None)
    o = L.mvgs_options()
    o.alloc = keep
    h = C.c_void_p()
    assert lib.mvgs_create(C.byref(h), C.byref(o)) == L.MVGS_EINVAL
    keep2 = L.FREE_FN(lambda p, c: None)
    o2 = L.mvgs_options()
    o2.free = keep2
    assert lib.mvgs_create(C.byref(h), C.byref(o2)) == L.MVGS_EINVAL


def _bound(lib, ctx, cams, P, rec, pairs, work=0):
    b = C.c_int64(-1)
    st = lib.mvgs_workspace_bound(ctx, L.camera_array(cams), len(cams), P, rec, pairs, work, C.byref(b))
    return st, b.value


def test_workspace_bound_is_host_only_and_monotone(ctx):
    """mvgs_workspace_bound does no device work: on a fresh context it is the sum of the grown sizes
    of every buffer the calls would make; it rises with records, pairs, views and the work asked for."""
    lib = L.lib()
    cams = scenes.make_cameras([(320, 180), (640, 480)])
    P = 100_000
    st, base = _bound(lib, ctx, cams, P, 1000, 5000)
    assert st == L.MVGS_OK and base > 0
    # records: at least a 64-byte blend record, view, keys, values and rectangles each (double-buffered)
    assert _bound(lib, ctx, cams, P, 101_000, 5000)[1] - base >= 100_000 * (64 + 2 + 4 * 4 + 8 * 2)
    # pairs: keys and values, double-buffered
    assert _bound(lib, ctx, cams, P, 1000, 1_005_000)[1] - base >= 1_000_000 * 16
    assert _bound(lib, ctx, cams[:1], P, 1000, 5000)[1] < base
    l1 = _bound(lib, ctx, cams, P, 1000, 5000, L.MVGS_WORK_LOSS)[1]
    ds = _bound(lib, ctx, cams, P, 1000, 5000, L.MVGS_WORK_LOSS_DSSIM)[1]
    bw = _bound(lib, ctx, cams, P, 1000, 5000, L.MVGS_WORK_LOSS_DSSIM | L.MVGS_WORK_BACKWARD)[1]
    assert base < l1 <= ds < bw   # D-SSIM adds only partial sums (two per 32x32 tile and channel)
    # the backward adds 48 bytes of accumulators per record
    assert bw - ds >= 1000 * 48
    # the context holds nothing: the bound allocated nothing
    held = C.c_int64(-1)
    assert lib.mvgs_memory_held(ctx, C.byref(held)) == L.MVGS_OK and held.value == 0


def test_workspace_bound_rejects_impossible_counts(ctx):
    lib = L.lib()
    cams = scenes.make_cameras([(64, 64)])
    assert _bound(lib, ctx, cams, 100, 101, 5)[0] == L.MVGS_EINVAL     # more records than Gaussians x views
    assert _bound(lib, ctx, cams, 100, -1, 5)[0] == L.MVGS_EINVAL
    assert _bound(lib, ctx, cams, 100, 10, -5)[0] == L.MVGS_EINVAL
    assert _bound(lib, ctx, cams, 100, 10, 5, 8)[0] == L.MVGS_EINVAL   # unknown work flag
    assert _bound(lib, ctx, cams, 100, 10, 1 << 32)[0] == L.MVGS_ECAPACITY
    assert _bound(lib, ctx, [], 100, 0, 0)[0] == L.MVGS_EINVAL
    b = C.c_int64()
    assert lib.mvgs_workspace_bound(ctx, L.camera_array(cams), 1, 100, 1, 1, 0, None) == L.MVGS_EINVAL
    assert lib.mvgs_workspace_bound(None, L.camera_array(cams), 1, 100, 1, 1, 0, C.byref(b)) == L.MVGS_EINVAL


def test_count_views_validates_before_the_device(ctx):
    lib = L.lib()
    cams = scenes.make_cameras([(64, 64)])
    rec = np.zeros(1, np.int64)
    pairs = np.zeros(1, np.int64)
    g = L.mvgs_gaussians()
    g.P, g.sh_degree = 10, 5
    assert lib.mvgs_count_views(ctx, None, C.byref(g), L.camera_array(cams), 1, rec.ctypes.data,
                                pairs.ctypes.data) == L.MVGS_EINVAL
    g.sh_degree = 0
    assert lib.mvgs_count_views(ctx, None, C.byref(g), L.camera_array(cams), 1, rec.ctypes.data,
                                pairs.ctypes.data) == L.MVGS_EINVAL   # NULL parameter pointers
