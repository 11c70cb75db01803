"""Host-side checks of the C ABI: the library loads, exports every declared symbol,
and validates its arguments before touching any device memory (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

import workloads as W
from conftest import ROOT
from paper_1908_06742_amd import _lib as L


def declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(ddf_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.SIGNATURES), "binding and header disagree"


def _create(pr):
    p = L.params_from_problem(pr)
    h = C.c_void_p()
    # fake aligned addresses: validation fails before they are used
    rc = L.lib().ddf_create(C.byref(p), C.c_void_p(1 << 20), C.c_void_p(2 << 20), C.c_void_p(3 << 20), C.byref(h))
    msg = L.lib().ddf_last_error().decode()
    if rc == 0:
        L.lib().ddf_destroy(h)
    return rc, msg


@pytest.mark.parametrize("bad,needle", [
    (dict(beta2=1.0), "beta1 == beta2"),
    (dict(nx=1), "nx and ny"),
    (dict(tau=0.5), "(0, 2)"),
    (dict(tau_phi=0.49), "(0, 2)"),
    (dict(storage="f64", rho0=0.0), "rho0"),
])
def test_create_rejects_invalid_parameters(bad, needle):
    pr = W.taylor_green_problem(16).with_(**bad)
    rc, msg = _create(pr)
    assert rc == L.DDF_ERR_ARG and needle in msg


def test_largest_lattice_is_accepted_and_one_row_more_is_not():
    # 2^31 nodes is the limit; such a lattice takes the 64-bit lane offsets (an FP32
    # plane of 8 GiB) and its byte counts do not wrap
    lib = L.lib()
    for storage, s in (("f32", 4), ("bf16", 2)):
        pr = W.Problem(nx=65536, ny=32768, storage=storage)
        p = L.params_from_problem(pr)
        nb = lib.ddf_population_bytes(C.byref(p))
        assert nb >= 9 * (1 << 31) * s and nb % 256 == 0
        h = C.c_void_p()
        assert lib.ddf_create(C.byref(p), C.c_void_p(1 << 20), C.c_void_p(2 << 20), C.c_void_p(3 << 20), C.byref(h)) == 0
        try:
            assert lib.ddf_get_address_width(h) == 64
            assert lib.ddf_set_address_width(h, 32) == L.DDF_ERR_ARG
        finally:
            lib.ddf_destroy(h)
        rc, msg = _create(pr.with_(ny=32769))
        assert rc == L.DDF_ERR_ARG and "2^31" in msg


def test_create_rejects_non_power_of_two_scale():
    pr = W.taylor_green_problem(16, storage="f16")
    pr.pop_scale = 3.0
    rc, msg = _create(pr)
    assert rc == L.DDF_ERR_ARG and "power of two" in msg


def test_create_rejects_unaligned_buffers():
    p = L.params_from_problem(W.taylor_green_problem(16))
    h = C.c_void_p()
    rc = L.lib().ddf_create(C.byref(p), C.c_void_p(1 << 20 | 8), C.c_void_p(2 << 20), C.c_void_p(3 << 20), C.byref(h))
    assert rc == L.DDF_ERR_ARG and "aligned" in L.lib().ddf_last_error().decode()


def test_valid_create_and_sizes():
    for storage, s in (("f64", 8), ("f32", 4), ("f16", 2), ("bf16", 2), ("bf16sr", 2)):
        pr = W.Problem(nx=100, ny=37, storage=storage)
        p = L.params_from_problem(pr)
        pitch = L.lib().ddf_pitch(C.byref(p))
        assert pitch == 128
        nb = L.lib().ddf_population_bytes(C.byref(p))
        assert nb >= 9 * pitch * 37 * s and nb % 256 == 0
        assert L.lib().ddf_workspace_bytes(C.byref(p)) > 3 * 100 * 37 * 4
        rc, msg = _create(pr)
        assert rc == 0, msg


def test_address_width_follows_the_plane_size():
    lib = L.lib()
    for pr, default in ((W.taylor_green_problem(16), 32), (W.Problem(nx=24000, ny=24000, storage="f64"), 64)):
        p = L.params_from_problem(pr)
        h = C.c_void_p()
        assert lib.ddf_create(C.byref(p), C.c_void_p(1 << 20), C.c_void_p(2 << 20), C.c_void_p(3 << 20), C.byref(h)) == 0
        try:
            assert lib.ddf_get_address_width(h) == default
            assert lib.ddf_set_address_width(h, 64) == 0 and lib.ddf_get_address_width(h) == 64
            rc = lib.ddf_set_address_width(h, 32)
            if default == 32:
                assert rc == 0 and lib.ddf_get_address_width(h) == 32
            else:
                assert rc == L.DDF_ERR_ARG and "4 GiB" in lib.ddf_last_error().decode()
                assert lib.ddf_get_address_width(h) == 64
            assert lib.ddf_set_address_width(h, 48) == L.DDF_ERR_ARG
        finally:
            lib.ddf_destroy(h)
    assert lib.ddf_set_address_width(None, 32) == L.DDF_ERR_ARG


def test_workgroup_caps_default_by_storage_and_size():
    lib = L.lib()
    cav = lambda n, storage: W.cavity_problem(n, 1000.0, 0.1, storage=storage)
    per = lambda n, storage: W.Problem(nx=n, ny=n, storage=storage)
    # 8192^2: x-interleaved rows; 8000^2: row-major rows; 1024^2: held by the cache
    cases = [(per, "f32", 8192, (2, 2), 32), (per, "f16", 8192, (3, 3), 64), (per, "bf16", 8192, (3, 0), 64),
             (per, "bf16sr", 8192, (3, 0), 32), (per, "f64", 8192, (1, 1), 32), (per, "f32", 1024, (0, 0), 32),
             (cav, "f32", 8192, (2, 2), 32), (cav, "f16", 8192, (3, 0), 32), (cav, "f64", 8192, (1, 1), 32),
             (per, "f64", 1024, (0, 0), 32),
             (per, "f32", 8000, (1, 1), 32), (per, "f16", 8000, (3, 2), 64), (per, "bf16sr", 8000, (0, 0), 32),
             (cav, "f32", 8000, (2, 2), 32), (cav, "f16", 8000, (0, 0), 32), (per, "f64", 8000, (1, 1), 32)]
    for make, storage, n, caps, bits in cases:
        p = L.params_from_problem(make(n, storage))
        h = C.c_void_p()
        assert lib.ddf_create(C.byref(p), C.c_void_p(1 << 20), C.c_void_p(2 << 20), C.c_void_p(3 << 20), C.byref(h)) == 0
        try:
            e, o = C.c_int32(), C.c_int32()
            assert lib.ddf_get_workgroups_per_cu(h, C.byref(e), C.byref(o)) == 0
            assert (e.value, o.value) == caps, storage
            assert lib.ddf_get_address_width(h) == bits, storage
            in_cache = 2 * lib.ddf_population_bytes(C.byref(p)) <= 256 << 20
            want_tw = 512 if in_cache else (64 if storage in ("f16", "bf16", "bf16sr") else 128)
            assert lib.ddf_get_tile_width(h) == want_tw, (storage, n)
            assert lib.ddf_set_workgroups_per_cu(h, 3, 0) == 0
            assert lib.ddf_get_workgroups_per_cu(h, C.byref(e), C.byref(o)) == 0 and (e.value, o.value) == (3, 0)
            for bad in ((4, 0), (0, 4), (-1, 2)):
                assert lib.ddf_set_workgroups_per_cu(h, *bad) == L.DDF_ERR_ARG
            assert lib.ddf_get_workgroups_per_cu(h, None, C.byref(o)) == L.DDF_ERR_ARG
        finally:
            lib.ddf_destroy(h)


def test_step_before_init_is_a_state_error():
    p = L.params_from_problem(W.taylor_green_problem(16))
    h = C.c_void_p()
    assert L.lib().ddf_create(C.byref(p), C.c_void_p(1 << 20), C.c_void_p(2 << 20), C.c_void_p(3 << 20), C.byref(h)) == 0
    try:
        assert L.lib().ddf_step(h, 1, None) == L.DDF_ERR_STATE
        assert L.lib().ddf_step(h, -1, None) == L.DDF_ERR_ARG
        buf = (C.c_double * 8)()
        assert L.lib().ddf_reduce(h, buf, None) == L.DDF_ERR_STATE
    finally:
        L.lib().ddf_destroy(h)


def test_weight_gradient_rejects_bad_arguments_before_any_launch():
    lib = L.lib()
    a, b, w = C.c_void_p(1 << 20), C.c_void_p(2 << 20), C.c_void_p(3 << 20)
    dw, db = C.cast(C.c_void_p(4 << 20), C.POINTER(C.c_float)), C.cast(C.c_void_p(5 << 20), C.POINTER(C.c_float))
    cases = [
        ((a, 1, 8, 8, 32, 32, 0, b, 32, 32, dw, db, 0, C.c_void_p(3 << 20 | 4), None), "aligned"),
        ((C.c_void_p(1 << 20 | 8), 1, 8, 8, 32, 32, 0, b, 32, 32, dw, db, 0, w, None), "aligned"),
        ((a, 1, 8, 8, 48, 48, 0, b, 32, 32, dw, db, 0, w, None), "multiples of 32"),
        ((a, 1, 8, 8, 32, 32, 0, b, 288, 288, dw, db, 0, w, None), "at most 256"),
        ((a, 1, 8, 8, 32, 36, 0, b, 32, 32, dw, db, 0, w, None), "multiples of 8"),
    ]
    for args, needle in cases:
        assert lib.ddf_nn_conv3x3_wgrad(*args) == L.DDF_ERR_ARG
        assert needle in lib.ddf_last_error().decode()


@pytest.mark.parametrize("N,H,W,Cin,Cout,pixels_per_strip,strips", [
    (8, 256, 256, 32, 32, 128 * 8, 8 * 2 * 32),      # 128-pixel columns, strips of 8 rows: 512 workgroups
    (8, 256, 256, 96, 32, 128 * 32, 8 * 2 * 8),      # three channel tiles: 32 rows, 384 workgroups
    (8, 128, 128, 192, 64, 128 * 32, 8 * 1 * 4),     # twelve tiles: 32 rows, 384 workgroups
    (8, 64, 64, 384, 128, 64 * 64, 8 * 1 * 1),       # 64-pixel columns, 48 tiles: whole images, 384 workgroups
    (1, 4, 64, 64, 64, 64 * 4, 1),                   # a strip no taller than the image
    (2, 683, 192, 64, 32, 64 * 32, 2 * 3 * 22),      # 64-pixel columns (192 is no multiple of 128), ragged strips
])
def test_row_streaming_weight_gradient_plan(N, H, W, Cin, Cout, pixels_per_strip, strips):
    # Widths that are multiples of 64 take the row-streaming weight gradient: strips of 8,
    # 16, 32, ... rows, the shortest that leave at most 512 workgroups (one per strip and
    # 32 x 32 channel tile).  Its workspace holds one set of weight and bias partials per
    # strip.
    chunk = C.c_int32()
    nbytes = L.lib().ddf_nn_wgrad_workspace_bytes(N, H, W, Cin, Cout, C.byref(chunk))
    assert chunk.value == pixels_per_strip
    assert nbytes == strips * (9 * Cout * Cin + Cout) * 4


def test_cast_weights_multi_rejects_bad_tables_before_any_launch():
    lib = L.lib()
    ok = L.CastLayer(1 << 20, 2 << 20, 3 << 20, 32, 32, 32, 32)
    for n in (0, L.NN_CAST_MAX_LAYERS + 1):
        arr = (L.CastLayer * max(n, 1))(*([ok] * max(n, 1)))
        assert lib.ddf_nn_cast_weights_multi(n, arr, None) == L.DDF_ERR_ARG
    for bad in (L.CastLayer(None, 2 << 20, None, 32, 32, 32, 32), L.CastLayer(1 << 20, 2 << 20, None, 64, 32, 32, 32)):
        arr = (L.CastLayer * 2)(ok, bad)
        assert lib.ddf_nn_cast_weights_multi(2, arr, None) == L.DDF_ERR_ARG
        assert "layer 1" in lib.ddf_last_error().decode()


def test_batch_step_reduce_rejects_bad_arguments_before_any_launch():
    lib = L.lib()
    buf = (C.c_double * 8)()
    assert lib.ddf_batch_step_reduce(None, 2, buf, None) == L.DDF_ERR_ARG
    assert "NULL" in lib.ddf_last_error().decode()


@pytest.mark.parametrize("args,needle", [
    ((3, 4, 0, 1 << 20, 2 << 20, 1 << 20), "kind"),
    ((0, 3, 0, 1 << 20, 2 << 20, 1 << 20), "unroll"),
    ((0, 4, 0, 1 << 20, 2 << 20, 1000), "multiple of 16"),
    ((0, 4, 0, 1 << 20, 2 << 20, 0), "multiple of 16"),
    ((0, 4, 0, None, 2 << 20, 1 << 20), "src is NULL"),
    ((2, 4, 0, None, None, 1 << 20), "dst is NULL"),
    ((0, 4, 0, (1 << 20) + 8, 2 << 20, 1 << 20), "aligned"),
    ((0, 4, 0, 1 << 20, (1 << 20) + 4096, 1 << 20), "overlap"),
])
def test_bandwidth_probe_rejects_invalid_arguments(args, needle):
    kind, unroll, nt, src, dst, nbytes = args
    rc = L.lib().ddf_bandwidth_probe(kind, unroll, nt, src, dst, nbytes, None)
    assert rc == L.DDF_ERR_ARG and needle in L.lib().ddf_last_error().decode()


def test_pattern_probe_rejects_invalid_arguments_before_any_launch():
    lib = L.lib()
    assert lib.ddf_pattern_probe(None, 0, 0, None) == L.DDF_ERR_ARG
    assert "NULL" in lib.ddf_last_error().decode()
    assert lib.ddf_batch_pattern_probe(None, 0, None) == L.DDF_ERR_ARG
    assert "NULL" in lib.ddf_last_error().decode()
    for pr, cases in ((W.taylor_green_problem(16), ((2, 0, L.DDF_ERR_ARG, "parity"), (1, 4, L.DDF_ERR_ARG, "per CU"),
                                                    (0, -1, L.DDF_ERR_ARG, "per CU"))),
                      (W.Problem(nx=16, ny=16, periodic_x=False, periodic_y=False), ((-1, 1, L.DDF_ERR_ARG, "parity"),))):
        p = L.params_from_problem(pr)
        h = C.c_void_p()
        assert lib.ddf_create(C.byref(p), C.c_void_p(1 << 20), C.c_void_p(2 << 20), C.c_void_p(3 << 20), C.byref(h)) == 0
        try:
            for parity, cap, rc, needle in cases:
                assert lib.ddf_pattern_probe(h, parity, cap, None) == rc
                assert needle in lib.ddf_last_error().decode()
        finally:
            lib.ddf_destroy(h)


def _create_rc(pr):
    p = L.params_from_problem(pr)
    h = C.c_void_p()
    rc = L.lib().ddf_create(C.byref(p), C.c_void_p(1 << 20), C.c_void_p(2 << 20), C.c_void_p(3 << 20), C.byref(h))
    layout = L.lib().ddf_get_layout(h) if rc == 0 else None
    if rc == 0:
        L.lib().ddf_destroy(h)
    return rc, layout


@pytest.mark.parametrize("storage,nx,ok", [
    ("f64", 1024, True), ("f64", 512, False), ("f32", 2048, True), ("f32", 1024, False), ("f32", 3072, False),
    ("f16", 4096, True), ("bf16", 2048, False), ("bf16sr", 8192, True), ("f32", 2000, False),
])
def test_interleaved_rows_need_a_power_of_two_width_of_whole_lines(storage, nx, ok):
    # nx = 64 * 2^k and nx / 64 at least one 128-byte line of the storage type
    rc, layout = _create_rc(W.Problem(nx=nx, ny=4, storage=storage, layout="interleaved"))
    if ok:
        assert rc == L.DDF_OK and layout == 2
    else:
        assert rc == L.DDF_ERR_UNSUPPORTED and "x-interleaved" in L.lib().ddf_last_error().decode()
    rc, layout = _create_rc(W.Problem(nx=nx, ny=4, storage=storage, layout="row"))
    assert rc == L.DDF_OK and layout == 1


def test_automatic_layout_interleaves_only_lattices_beyond_the_cache():
    # two population arrays above 256 MB stream from HBM and take interleaved rows
    assert _create_rc(W.Problem(nx=8192, ny=8192, storage="f32"))[1] == 2
    assert _create_rc(W.Problem(nx=8192, ny=8192, storage="bf16"))[1] == 2
    assert _create_rc(W.Problem(nx=2048, ny=64, storage="f32"))[1] == 1       # in the cache
    assert _create_rc(W.Problem(nx=8000, ny=8000, storage="f32"))[1] == 1     # width not 64 * 2^k
    assert _create_rc(W.Problem(nx=32768, ny=32832, storage="f32"))[1] == 2   # 64-bit offsets


@pytest.mark.parametrize("layout", ["interleaved", "row"])
def test_batches_keep_packed_rows(layout):
    ps = (L.Params * 1)(L.params_from_problem(W.Problem(nx=2048, ny=4, storage="f32", layout=layout)))
    h = C.c_void_p()
    rc = L.lib().ddf_batch_create(1, ps, C.c_void_p(1 << 20), C.c_void_p(2 << 20), C.c_void_p(3 << 20), C.byref(h))
    assert rc == L.DDF_ERR_UNSUPPORTED and "packed rows" in L.lib().ddf_last_error().decode()
    assert L.lib().ddf_batch_workspace_bytes(1, ps) == 0


@pytest.mark.parametrize("storage,s", [("f64", 8), ("f32", 4), ("f16", 2), ("bf16sr", 2)])
def test_packed_rows_drop_the_row_padding(storage, s):
    lib = L.lib()
    for nx, ny in ((77, 5), (131, 37), (64, 3), (2, 2)):
        row = L.params_from_problem(W.Problem(nx=nx, ny=ny, storage=storage, layout="row"))
        pk = L.params_from_problem(W.Problem(nx=nx, ny=ny, storage=storage, layout="packed"))
        assert lib.ddf_pitch(C.byref(row)) == (nx + 63) // 64 * 64
        assert lib.ddf_pitch(C.byref(pk)) == nx
        plane = lib.ddf_plane_stride(C.byref(pk))
        assert plane == (nx * ny + 63) // 64 * 64          # every plane starts on a 128-byte line
        assert lib.ddf_population_bytes(C.byref(pk)) == (9 * plane * s + 255) // 256 * 256
        assert _create_rc(W.Problem(nx=nx, ny=ny, storage=storage, layout="packed")) == (L.DDF_OK, 3)
    # a batch lays its instances out as packed rows, whatever layout AUTO would give alone
    probs = [W.Problem(nx=77, ny=5, storage=storage), W.Problem(nx=8192, ny=8192, storage=storage)]
    ps = (L.Params * 2)(*[L.params_from_problem(p) for p in probs])
    want = sum(lib.ddf_population_bytes(C.byref(L.params_from_problem(p.with_(layout="packed")))) for p in probs)
    assert lib.ddf_batch_population_bytes(2, ps) == want
