"""The C-ABI library loads, exports every entry point include/*.h declares, and
rejects bad arguments on the host before touching a device (no GPU needed:
validation runs before the context is looked at, so a NULL context is enough)."""
import ctypes
import glob
import os
import re

import pytest

from paper_2601_00551_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(sbp\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("sbp_simulate_signals", "sbp_adjoint_gradients", "sbp_filter_zero_grad",
                     "sbp_step", "sbp_downsample", "sbp_grow", "sbp_ctx_create", "sbp_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _abi.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding knows the signature of each
    assert set(declared_functions()) <= set(_abi.SIGNATURES)


def _model(**kw):
    m = _abi.SbpModel(1.5, 0.025, 0.0, 5.0, 512, 1, 1, 1, 0, 0)
    for k, v in kw.items():
        setattr(m, k, v)
    return m


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


def _array(D=4):
    return _abi.SbpArray(FAKE.value, FAKE.value, FAKE.value, FAKE.value, FAKE.value, FAKE.value, D, 0)


def _balls():
    return _abi.SbpBalls(FAKE.value, FAKE.value, FAKE.value, FAKE.value, FAKE.value)


def _sim(ctx=None, arr=None, balls=None, off=FAKE, F=1, cap=10, model=None, y=FAKE, acc=0,
         fn="sbp_simulate_signals"):
    return getattr(_abi.lib(), fn)(ctx, ctypes.byref(arr or _array()), ctypes.byref(balls or _balls()),
                                   off, F, cap, ctypes.byref(model or _model()), y, acc, None)


def last():
    return _abi.lib().sbp_last_error().decode()


@pytest.mark.parametrize("kw,code", [
    (dict(model=_model(c=0.0)), _abi.SBP_E_DOMAIN),
    (dict(model=_model(c=-1.5)), _abi.SBP_E_DOMAIN),
    (dict(model=_model(dt=0.0)), _abi.SBP_E_DOMAIN),
    (dict(model=_model(f=0)), _abi.SBP_E_DOMAIN),
    (dict(model=_model(T=0)), _abi.SBP_E_DOMAIN),
    (dict(model=_model(profile=7)), _abi.SBP_E_DOMAIN),
    (dict(model=_model(directivity=-1)), _abi.SBP_E_DOMAIN),
    (dict(model=_model(gauss_K=0.0)), _abi.SBP_E_DOMAIN),
    (dict(model=_model(gauss_K=12.5)), _abi.SBP_E_DOMAIN),
    (dict(model=_model(gauss_K=float("inf"))), _abi.SBP_E_DOMAIN),
    (dict(model=_model(a_softplus=2)), _abi.SBP_E_DOMAIN),
    (dict(model=_model(t0=float("nan"))), _abi.SBP_E_DOMAIN),
    (dict(F=0), _abi.SBP_E_ARG),
    (dict(F=65), _abi.SBP_E_ARG),
    (dict(cap=-1), _abi.SBP_E_ARG),
    (dict(off=None), _abi.SBP_E_ARG),
    (dict(y=None), _abi.SBP_E_ARG),
    (dict(acc=3), _abi.SBP_E_ARG),
    (dict(arr=_array(D=0)), _abi.SBP_E_ARG),
    (dict(balls=_abi.SbpBalls(FAKE.value, None, FAKE.value, FAKE.value, FAKE.value)), _abi.SBP_E_ARG),
    (dict(), _abi.SBP_E_ARG),          # everything valid but the NULL context
])
@pytest.mark.parametrize("fn", ["sbp_simulate_signals", "sbp_simulate_signals_noalloc"])
def test_simulate_validation(kw, code, fn):
    assert _sim(fn=fn, **kw) == code
    assert last()


def test_noalloc_rejects_workspace_beyond_its_fixed_size():
    """The allocation-free forward's fixed workspace is 128 MiB per GPU: a call
    needing more (8 (T + 1) F D + 24 B_cap bytes) is refused on the host,
    before the context is looked at, with the sizes in the message."""
    fn = "sbp_simulate_signals_noalloc"
    # 1024 transducers x 20000 samples: 164 MB of per-sample sums
    assert _sim(fn=fn, arr=_array(D=1024), model=_model(T=20000)) == _abi.SBP_E_CAPACITY
    assert "the fixed workspace holds %d" % ((128 << 20) - 512) in last(), last()
    # 6,000,000 balls: 144 MB of per-ball constants
    assert _sim(fn=fn, cap=6_000_000) == _abi.SBP_E_CAPACITY
    # the large workload of the benchmark fits: 1024 x 4097 x 8 + 24 x 2,000,000 bytes
    assert _sim(fn=fn, arr=_array(D=1024), model=_model(T=4096), cap=2_000_000) == _abi.SBP_E_ARG
    assert "ctx" in last()


def test_uniform_profile_ignores_gauss_K():
    # gauss_K is only checked for the GAUSS profile; with the NULL context last
    assert _sim(model=_model(profile=0, gauss_K=0.0)) == _abi.SBP_E_ARG
    assert "ctx" in last()


def test_adjoint_validation():
    lib = _abi.lib()
    g = _balls()
    call = lambda mask, grad=g, v=FAKE, model=None: lib.sbp_adjoint_gradients(
        None, ctypes.byref(_array()), ctypes.byref(_balls()), FAKE, 1, 10,
        ctypes.byref(model or _model()), v, mask, ctypes.byref(grad), None)
    assert call(0) == _abi.SBP_E_ARG
    assert call(64) == _abi.SBP_E_ARG
    assert call(_abi.ALL, v=None) == _abi.SBP_E_ARG
    g2 = _abi.SbpBalls(None, None, None, FAKE.value, None)
    assert call(_abi.P0, grad=g2) == _abi.SBP_E_ARG and "ctx" in last()   # p0-only with others NULL is fine
    assert call(_abi.ALL, grad=g2) == _abi.SBP_E_ARG and "grad" in last()
    assert call(_abi.ALL, model=_model(f=-2)) == _abi.SBP_E_DOMAIN
    assert call(_abi.ALL, model=_model(sampling=7)) == _abi.SBP_E_DOMAIN and "sampling" in last()
    # point sampling exists for the GAUSS profile only
    assert call(_abi.ALL, model=_model(sampling=_abi.SAMPLING_POINT, profile=0)) == _abi.SBP_E_DOMAIN
    assert "GAUSS" in last()
    assert call(_abi.ALL, model=_model(sampling=_abi.SAMPLING_POINT)) == _abi.SBP_E_ARG   # then ctx


def test_downsample_validation():
    lib = _abi.lib()
    assert lib.sbp_downsample(None, FAKE, 4, 100, 0, FAKE, None) == _abi.SBP_E_DOMAIN
    assert lib.sbp_downsample(None, FAKE, 4, 3, 4, FAKE, None) == _abi.SBP_E_DOMAIN
    assert lib.sbp_downsample(None, FAKE, 0, 100, 2, FAKE, None) == _abi.SBP_E_ARG
    assert lib.sbp_downsample(None, None, 4, 100, 2, FAKE, None) == _abi.SBP_E_ARG
    assert lib.sbp_downsample(None, FAKE, 4, 100, 2, FAKE, None) == _abi.SBP_E_ARG
    assert "ctx" in last()


def test_decimate_validation():
    lib = _abi.lib()
    assert lib.sbp_decimate(None, FAKE, 4, 100, 0, FAKE, None) == _abi.SBP_E_DOMAIN
    assert lib.sbp_decimate(None, FAKE, 4, 3, 4, FAKE, None) == _abi.SBP_E_DOMAIN
    assert lib.sbp_decimate(None, FAKE, 0, 100, 2, FAKE, None) == _abi.SBP_E_ARG
    assert lib.sbp_decimate(None, FAKE, 4, 100, 2, None, None) == _abi.SBP_E_ARG
    assert lib.sbp_decimate(None, FAKE, 4, 100, 2, FAKE, None) == _abi.SBP_E_ARG
    assert "ctx" in last()


def test_filter_validation():
    lib = _abi.lib()
    b = _balls()

    def call(strict=1, m_in=None, y_ref=FAKE, off_out=FAKE):
        return lib.sbp_filter_zero_grad(None, ctypes.byref(_array()), ctypes.byref(b), FAKE, 1, 10,
                                        ctypes.byref(_model()), y_ref, strict, ctypes.byref(b), off_out,
                                        None, m_in, None, None, None, None)
    assert call(strict=2) == _abi.SBP_E_ARG
    assert call(y_ref=None) == _abi.SBP_E_ARG
    assert call(off_out=None) == _abi.SBP_E_ARG
    assert call(m_in=ctypes.byref(b)) == _abi.SBP_E_ARG and "v_in" in last()  # moments all or none
    assert call() == _abi.SBP_E_ARG and "ctx" in last()


def test_adam_and_step_validation():
    lib = _abi.lib()
    st = _abi.SbpState(_balls(), _balls(), _balls(), _balls(), FAKE.value, 1, 0, 10)
    p = _abi.SbpAdamParams((ctypes.c_float * 5)(0.1, 0.1, 0.1, 0.1, 0.1), 0.9, 0.999, 1e-8, 1, _abi.ALL)
    assert lib.sbp_adam_update(None, ctypes.byref(st), ctypes.byref(p), None, None) == _abi.SBP_E_ARG
    assert "ctx" in last()
    bad = _abi.SbpAdamParams((ctypes.c_float * 5)(0.1, 0.1, 0.1, 0.1, 0.1), 1.0, 0.999, 1e-8, 1, _abi.ALL)
    assert lib.sbp_adam_update(None, ctypes.byref(st), ctypes.byref(bad), None, None) == _abi.SBP_E_DOMAIN
    zero_step = _abi.SbpAdamParams((ctypes.c_float * 5)(0.1, 0.1, 0.1, 0.1, 0.1), 0.9, 0.999, 1e-8, 0, _abi.ALL)
    assert lib.sbp_adam_update(None, ctypes.byref(st), ctypes.byref(zero_step), None, None) == _abi.SBP_E_DOMAIN
    # with a device step counter the host step is not used
    assert lib.sbp_adam_update(None, ctypes.byref(st), ctypes.byref(zero_step), FAKE, None) == _abi.SBP_E_ARG
    st_nog = _abi.SbpState(_balls(), _abi.SbpBalls(), _balls(), _balls(), FAKE.value, 1, 0, 10)
    assert lib.sbp_adam_update(None, ctypes.byref(st_nog), ctypes.byref(p), None, None) == _abi.SBP_E_ARG
    assert "grad" in last()
    assert lib.sbp_step(None, ctypes.byref(_array()), ctypes.byref(st), ctypes.byref(_model()), FAKE, FAKE,
                        ctypes.byref(p), None, None) == _abi.SBP_E_ARG
    assert lib.sbp_step(None, ctypes.byref(_array()), ctypes.byref(st), ctypes.byref(_model(T=-1)), FAKE, FAKE,
                        ctypes.byref(p), FAKE, None) == _abi.SBP_E_DOMAIN


def test_grow_and_graph_validation():
    lib = _abi.lib()
    st = _abi.SbpState(_balls(), _balls(), _balls(), _balls(), FAKE.value, 1, 0, 10)
    st2 = _abi.SbpState(_balls(), _balls(), _balls(), _balls(), FAKE.value, 2, 0, 10)
    rule = _abi.SbpGrowthRule(0.02, 0.02, 0.3, 0.1, 0.5, 0)
    cnt = ctypes.c_int64()
    assert lib.sbp_grow(None, ctypes.byref(st), ctypes.byref(rule), ctypes.byref(st2), ctypes.byref(cnt), None) == _abi.SBP_E_ARG
    assert "F" in last()
    bad = _abi.SbpGrowthRule(0.02, 0.02, 0.3, 1.5, 0.5, 0)
    assert lib.sbp_grow(None, ctypes.byref(st), ctypes.byref(bad), ctypes.byref(st), ctypes.byref(cnt), None) == _abi.SBP_E_DOMAIN
    assert lib.sbp_grow(None, ctypes.byref(st), ctypes.byref(rule), ctypes.byref(st), ctypes.byref(cnt), None) == _abi.SBP_E_ARG
    assert "ctx" in last()
    p = _abi.SbpAdamParams((ctypes.c_float * 5)(0.1, 0.1, 0.1, 0.1, 0.1), 0.9, 0.999, 1e-8, 1, _abi.ALL)
    g = ctypes.c_void_p()
    assert lib.sbp_step_graph_create(None, ctypes.byref(_array()), ctypes.byref(st), ctypes.byref(_model()),
                                     FAKE, FAKE, ctypes.byref(p), FAKE, FAKE, 0, ctypes.byref(g), FAKE) == _abi.SBP_E_ARG
    assert lib.sbp_step_graph_create(None, ctypes.byref(_array()), ctypes.byref(st), ctypes.byref(_model()),
                                     FAKE, FAKE, ctypes.byref(p), FAKE, FAKE, 2, ctypes.byref(g), None) == _abi.SBP_E_ARG
    assert "stream" in last()
    assert lib.sbp_graph_launch(None, None) == _abi.SBP_E_ARG
    assert lib.sbp_graph_destroy(None) == _abi.SBP_OK
    assert lib.sbp_ctx_destroy(None) == _abi.SBP_OK


def test_tuning_validation():
    lib = _abi.lib()
    t = _abi.SbpTuning(4, 512, 2, 0, 4, 256, 2, 0)
    assert lib.sbp_ctx_set_tuning(None, ctypes.byref(t)) == _abi.SBP_E_ARG and "ctx" in last()
    for field, val in (("fwd_dets", 0), ("fwd_dets", 17), ("fwd_block", 100), ("adj_bpt", 4), ("adj_grid", -1),
                       ("fwd_tile", 10), ("adj_tile", -1)):
        bad = _abi.SbpTuning(4, 512, 2, 0, 4, 256, 2, 0)
        setattr(bad, field, val)
        assert lib.sbp_ctx_set_tuning(None, ctypes.byref(bad)) == _abi.SBP_E_DOMAIN, field


def test_context_create_rejects_bad_device():
    lib = _abi.lib()
    p = ctypes.c_void_p()
    assert lib.sbp_ctx_create(ctypes.byref(p), -1) == _abi.SBP_E_ARG
    assert lib.sbp_ctx_create(None, 0) == _abi.SBP_E_ARG


def test_image_entry_points_validate_on_the_host():
    lib = _abi.lib()
    d = ctypes.c_void_p(256)
    assert lib.sbp_image_metrics(None, d, d, 10, 20, 20, 1.0, d, d, None) == _abi.SBP_E_DOMAIN
    assert lib.sbp_image_metrics(None, d, d, 20, 20, 20, 0.0, d, d, None) == _abi.SBP_E_DOMAIN
    assert lib.sbp_image_metrics(None, d, d, 20, 20, 20, 1.0, d, d, None) == _abi.SBP_E_ARG
    assert lib.sbp_image_metrics(None, None, d, 20, 20, 20, 1.0, d, d, None) == _abi.SBP_E_ARG
    grid = _abi.SbpGrid(0.0, 0.0, 0.0, 0.0, 4, 4, 4, 0)
    model = _abi.SbpModel(1.5, 0.025, 0.0, 5.0, 100, 1, 1, 1, 0, 0)
    balls = _abi.SbpBalls(d, d, d, d, d)
    assert lib.sbp_voxelize(None, ctypes.byref(balls), d, 10, ctypes.byref(model), ctypes.byref(grid), d,
                            None) == _abi.SBP_E_DOMAIN


# ------------------------------------------------------- transducer response --

@pytest.mark.parametrize("kw,code", [
    (dict(response=FAKE.value, response_taps=0), _abi.SBP_E_DOMAIN),
    (dict(response=FAKE.value, response_taps=4096), _abi.SBP_E_DOMAIN),
    (dict(response=FAKE.value, response_taps=31, response_zero=-1), _abi.SBP_E_DOMAIN),
    (dict(response=FAKE.value, response_taps=31, response_zero=31), _abi.SBP_E_DOMAIN),
    (dict(response=FAKE.value, response_taps=31, response_zero=15, response_rows=3), _abi.SBP_E_ARG),
    (dict(reserved=1), _abi.SBP_E_ARG),
])
def test_model_response_fields_are_validated(kw, code):
    """The response fields of the model are checked on the host (rows against
    the array's D = 4) by every call that takes a model."""
    assert _sim(model=_model(**kw)) == code
    assert "response" in last() or "reserved" in last(), last()
    lib = _abi.lib()
    g = _balls()
    assert lib.sbp_adjoint_gradients(None, ctypes.byref(_array()), ctypes.byref(_balls()), FAKE, 1, 10,
                                     ctypes.byref(_model(**kw)), FAKE, _abi.ALL, ctypes.byref(g),
                                     None) == code


def test_model_with_a_valid_response_reaches_the_context_check():
    for rows in (1, 4):
        m = _model(response=FAKE.value, response_taps=31, response_zero=15, response_rows=rows)
        assert _sim(model=m) == _abi.SBP_E_ARG
        assert "ctx" in last()
    # with no taps pointer the other fields are ignored
    assert _sim(model=_model(response_taps=-3, response_rows=7)) == _abi.SBP_E_ARG
    assert "ctx" in last()


def test_noalloc_counts_the_response_record():
    fn = "sbp_simulate_signals_noalloc"
    resp = dict(response=FAKE.value, response_taps=31, response_zero=15, response_rows=1)
    # 1024 x 8000 samples and 2M balls fit without a response (113.5 MB) ...
    assert _sim(fn=fn, arr=_array(D=1024), model=_model(T=8000), cap=2_000_000) == _abi.SBP_E_ARG
    # ... but not with the 32.8 MB record before it
    assert _sim(fn=fn, arr=_array(D=1024), model=_model(T=8000, **resp), cap=2_000_000) == \
        _abi.SBP_E_CAPACITY


def test_response_length_matches_the_oracle():
    from oracle import response as oresp
    L, zero = _abi.I32(), _abi.I32()
    for fc, bw, dt, ns in [(2.02, 0.54, 0.025, 5.0), (2.02, 0.54, 0.1, 5.0), (1.9, 0.5, 0.05, 4.0),
                           (2.3, 0.6, 0.0125, 6.0)]:
        assert _abi.lib().sbp_response_length(fc, bw, dt, ns, ctypes.byref(L), ctypes.byref(zero)) == 0
        assert (L.value, zero.value) == oresp.taps_length(fc, bw, dt, ns)


@pytest.mark.parametrize("args,code", [
    ((0.0, 0.54, 0.025, 5.0), _abi.SBP_E_DOMAIN),
    ((2.02, -0.5, 0.025, 5.0), _abi.SBP_E_DOMAIN),
    ((2.02, 0.54, float("inf"), 5.0), _abi.SBP_E_DOMAIN),
    ((2.02, 0.54, 0.025, 0.0), _abi.SBP_E_DOMAIN),
    ((2.02, 0.54, 1e-5, 5.0), _abi.SBP_E_CAPACITY),
])
def test_response_length_validation(args, code):
    L, zero = _abi.I32(), _abi.I32()
    assert _abi.lib().sbp_response_length(*args, ctypes.byref(L), ctypes.byref(zero)) == code
    assert last()


@pytest.mark.parametrize("args,code", [
    (dict(fc=None), _abi.SBP_E_ARG),
    (dict(rows=0), _abi.SBP_E_ARG),
    (dict(dt=0.0), _abi.SBP_E_DOMAIN),
    (dict(L=0), _abi.SBP_E_DOMAIN),
    (dict(L=4096), _abi.SBP_E_DOMAIN),
    (dict(zero=31), _abi.SBP_E_DOMAIN),
    (dict(), _abi.SBP_E_ARG),         # valid but the NULL context
])
def test_response_taps_validation(args, code):
    a = dict(fc=FAKE, bw=FAKE, rows=4, dt=0.025, L=31, zero=15, h=FAKE)
    a.update(args)
    assert _abi.lib().sbp_response_taps(None, a["fc"], a["bw"], a["rows"], a["dt"], a["L"], a["zero"],
                                        a["h"], None) == code
    assert last()


@pytest.mark.parametrize("args,code", [
    (dict(h=None), _abi.SBP_E_ARG),
    (dict(R=0), _abi.SBP_E_ARG),
    (dict(rows_h=3), _abi.SBP_E_ARG),
    (dict(rows_h=4, R=6), _abi.SBP_E_ARG),
    (dict(adjoint=2), _abi.SBP_E_ARG),
    (dict(accumulate=-1), _abi.SBP_E_ARG),
    (dict(out=ctypes.c_void_p(0x1000 + 4 * 100)), _abi.SBP_E_ARG),    # overlaps y
    (dict(T=0), _abi.SBP_E_DOMAIN),
    (dict(L=0), _abi.SBP_E_DOMAIN),
    (dict(zero=-1), _abi.SBP_E_DOMAIN),
    (dict(out=ctypes.c_void_p(0x1000 + 4 * 8 * 64)), _abi.SBP_E_ARG),  # adjacent: the NULL context
])
def test_response_apply_validation(args, code):
    a = dict(h=FAKE, rows_h=1, L=31, zero=15, y=FAKE, R=8, D=4, T=64, adjoint=0, accumulate=0,
             out=ctypes.c_void_p(0x100000))
    a.update(args)
    rc = _abi.lib().sbp_response_apply(None, a["h"], a["rows_h"], a["L"], a["zero"], a["y"], a["R"],
                                       a["D"], a["T"], a["adjoint"], a["accumulate"], a["out"], None)
    assert rc == code
    assert last()


# -------------------------------------------------- multi-frame proposals --

def _state_struct(F=2, cap=10, null_off=False):
    b = _balls()
    return _abi.SbpState(b, _abi.SbpBalls(), _abi.SbpBalls(), _abi.SbpBalls(), None if null_off else FAKE.value,
                         F, 0, cap)


@pytest.mark.parametrize("kw,code", [
    (dict(site_off=None), _abi.SBP_E_ARG),
    (dict(scale=None), _abi.SBP_E_ARG),
    (dict(M=-1), _abi.SBP_E_ARG),
    (dict(out=None), _abi.SBP_E_ARG),                     # M > 0 needs the outputs
    (dict(in_F=0), _abi.SBP_E_ARG),
    (dict(in_F=65, out_F=65), _abi.SBP_E_ARG),
    (dict(out_F=3), _abi.SBP_E_ARG),                      # frame counts differ
    (dict(null_off=True), _abi.SBP_E_ARG),
    (dict(a_init=0.0), _abi.SBP_E_DOMAIN),
    (dict(), _abi.SBP_E_ARG),                             # valid but the NULL context
])
def test_merge_proposals_validation(kw, code):
    a = dict(site_off=FAKE, scale=FAKE, M=5, out=FAKE, in_F=2, out_F=2, null_off=False, a_init=0.1)
    a.update(kw)
    s_in = _state_struct(a["in_F"], null_off=a["null_off"])
    s_out = _state_struct(a["out_F"])
    cnt = ctypes.c_int64()
    rc = _abi.lib().sbp_merge_proposals(None, ctypes.byref(s_in), ctypes.byref(_balls()), a["site_off"],
                                        a["out"], a["M"], a["scale"], a["a_init"], ctypes.byref(s_out),
                                        ctypes.byref(cnt), None)
    assert rc == code
    assert last()
