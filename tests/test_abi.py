"""The C ABI on the host: the library loads, exports every function that
include/apsm.h declares, and rejects invalid arguments before touching the
device (so these run without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_2201_05024_amd as A

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "apsm.h")

needs_lib = pytest.mark.skipif(not os.path.exists(A.LIB_PATH),
                               reason="libapsm.so not built (run python -m paper_2201_05024_amd.build)")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(apsm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("apsm_train", "apsm_detect", "apsm_get_status", "apsm_strerror",
                     "apsm_last_hip_error", "apsm_version"):
        assert required in names


@needs_lib
def test_every_declared_symbol_is_exported():
    L = A.library()
    for name in declared_functions():
        assert hasattr(L, name), name


@needs_lib
def test_strerror_and_version():
    L = A.library()
    assert L.apsm_version().decode().count(".") == 2
    for code in range(0, 8):
        assert isinstance(L.apsm_strerror(code), bytes) and L.apsm_strerror(code)
    assert L.apsm_strerror(A.ERR_WORKSPACE) != L.apsm_strerror(99)
    assert L.apsm_strerror(A.ERR_NONFINITE) != L.apsm_strerror(99)
    assert L.apsm_strerror(7) == L.apsm_strerror(99)          # not a code


@needs_lib
def test_shutdown_is_callable_any_time():
    A.shutdown()
    A.shutdown()
    # the library still works on the host afterwards
    L = A.library()
    assert L.apsm_train(None, 32, 6, 64, 1, 1, None, None) == A.ERR_INVALID_ARG


def _model(M2=32, K=6, cap=256, ptr=1, packed=1):
    return A._CModel(M2, K, cap, 0, ptr, ptr, ptr, ptr, packed)


def _params(**kw):
    base = dict(sigma2=0.5, eps=0.05, mu=1.0, w_lin=0.5, w_gauss=0.5, window=16, dict_cap=256,
                init=0, pos_weights=None, weights=0, extrapolate=0)
    base.update(kw)
    return A._CParams(**base)


BAD_TRAIN = [
    (dict(sigma2=0.0), 1), (dict(sigma2=float("nan")), 1), (dict(eps=-0.1), 1),
    (dict(mu=0.0), 1), (dict(mu=2.0), 1), (dict(w_lin=0.0, w_gauss=0.0), 1),
    (dict(w_lin=-1.0), 1), (dict(window=0), 1), (dict(window=65, dict_cap=256), 3),
    (dict(dict_cap=8, window=16), 1), (dict(extrapolate=2), 1), (dict(extrapolate=-1), 1),
    (dict(init=3), 1), (dict(init=-1), 1), (dict(init=1, w_lin=0.0, w_gauss=1.0), 1),
    (dict(init=2, w_lin=0.0, w_gauss=1.0), 1), (dict(weights=3), 1), (dict(weights=-1), 1),
]


@needs_lib
@pytest.mark.parametrize("kw,code", BAD_TRAIN)
def test_train_rejects_bad_params(kw, code):
    L = A.library()
    p = _params(**kw)
    cap = kw.get("dict_cap", 256)
    m = _model(cap=cap)
    assert L.apsm_train(ctypes.byref(p), 32, 6, 64, 1, 1, ctypes.byref(m), None) == code


@needs_lib
def test_train_rejects_bad_shapes_and_pointers():
    L = A.library()
    p = _params()
    m = _model()
    assert L.apsm_train(ctypes.byref(p), 32, 6, 64, None, 1, ctypes.byref(m), None) == 1
    assert L.apsm_train(None, 32, 6, 64, 1, 1, ctypes.byref(m), None) == 1
    assert L.apsm_train(ctypes.byref(p), 32, 6, 0, 1, 1, ctypes.byref(m), None) == 2
    assert L.apsm_train(ctypes.byref(p), 31, 6, 64, 1, 1, ctypes.byref(_model(M2=31)), None) == 2
    assert L.apsm_train(ctypes.byref(p), 32, 5, 64, 1, 1, ctypes.byref(m), None) == 2   # K mismatch
    assert L.apsm_train(ctypes.byref(p), 256, 6, 64, 1, 1, ctypes.byref(_model(M2=256)), None) == 3
    assert L.apsm_train(ctypes.byref(p), 32, 17, 64, 1, 1, ctypes.byref(_model(K=17)), None) == 3
    assert L.apsm_train(ctypes.byref(p), 32, 6, 64, 1, 1, ctypes.byref(_model(ptr=None)), None) == 1
    bad_w = (ctypes.c_float * 16)(*([1.0] * 15 + [0.0]))
    pw = _params(pos_weights=ctypes.cast(bad_w, ctypes.POINTER(ctypes.c_float)))
    assert L.apsm_train(ctypes.byref(pw), 32, 6, 64, 1, 1, ctypes.byref(m), None) == 1


@needs_lib
def test_detect_rejects_bad_args():
    L = A.library()
    m = _model()
    ok = dict(sigma2=0.5, S=10, rx=1, soft=1, hard=None, mod=0, truth=None, err=None)

    def call(**kw):
        a = dict(ok)
        a.update(kw)
        return L.apsm_detect(ctypes.byref(a.pop("model", m)), a["sigma2"], a["S"], a["rx"],
                             a["soft"], a["hard"], a["mod"], a["truth"], a["err"], None)

    assert call(sigma2=0.0) == 1
    assert call(S=-1) == 2
    assert call(mod=3) == 1
    assert call(hard=1, mod=0) == 1                     # decisions need a modulation
    assert call(truth=1, mod=2) == 1                    # truth without a counter
    assert call(soft=None) == 1                         # nothing to produce
    assert call(rx=None) == 1
    assert call(model=_model(M2=7)) == 2
    assert call(model=_model(K=0)) == 2
    assert call(model=_model(packed=None)) == 1         # every shape needs the packed form
    assert call(model=_model(M2=128, K=6, packed=None), S=0) == 1
    assert call(S=0) == 0                               # empty input: nothing launched
    assert call(S=0, rx=None, soft=None) == 0           # ... and no buffers needed


@needs_lib
def test_packed_bytes():
    L = A.library()
    L.apsm_model_packed_bytes.restype = ctypes.c_size_t
    def wide(m2p, cap):
        # two-contraction layout: 256-byte header, the linear weights (2M/32 x
        # 2 KiB), stages of 64 entries: the entries' hi and lo halves as
        # 1 KiB MFMA fragments (64 x 2M x 2 parts x 2 bytes), 4 KiB of
        # coefficients, 1 KiB of norms
        return 256 + m2p // 32 * 2048 + -(-cap // 64) * (64 * m2p * 2 * 2 + 4096 + 1024)

    def f16(m2p, k4, cap):
        # split-FP16 layout: 64-byte header, rows padded to 128 entries of
        # (2 * 2M + 8) halves and (K4 + 4) floats; the wide image follows at
        # the next multiple of 256 bytes
        return (64 + -(-cap // 128) * 128 * ((2 * m2p + 8) * 2 + (k4 + 4) * 4) + 255) // 256 * 256

    # 2M = 32, K = 6: both layouts (2M = 32 -> rows of (2*32 + 8) halves, K = 6 -> (8 + 4) floats per entry)
    assert L.apsm_model_packed_bytes(32, 6, 1000) == f16(32, 8, 1000) + wide(32, 1000)
    assert f16(32, 8, 1000) == (64 + 1024 * (72 * 2 + 12 * 4) + 255) // 256 * 256
    # two-contraction layout (2M > 64 or K > 8): 256-byte header, the linear
    # weights (2M/32 x 2 KiB), stages of 64 entries: hi and lo fragments of
    # 1 KiB (64 entries x 2M x 2 parts x 2 bytes), 4 KiB of coefficients,
    # 1 KiB of norms
    assert L.apsm_model_packed_bytes(128, 16, 1000) == 256 + 4 * 2048 + 16 * (32768 + 4096 + 1024)
    assert L.apsm_model_packed_bytes(128, 3, 64) == wide(128, 64)         # 2M > 64: one layout
    assert L.apsm_model_packed_bytes(32, 9, 65) == 256 + 1 * 2048 + 2 * (8192 + 4096 + 1024)
    assert L.apsm_model_packed_bytes(20, 12, 10) == L.apsm_model_packed_bytes(32, 16, 64)
    assert L.apsm_model_packed_bytes(66, 1, 10) == L.apsm_model_packed_bytes(128, 16, 64)
    # 2M = 40 runs with the 64-wide layouts: rows of 2*64+8 halves, K4 + 4 floats each
    assert L.apsm_model_packed_bytes(40, 2, 40) == f16(64, 4, 40) + wide(64, 40)
    for m2 in range(34, 65, 2):
        assert L.apsm_model_packed_bytes(m2, 5, 300) == L.apsm_model_packed_bytes(64, 5, 300), m2
    for m2 in range(18, 33, 2):
        assert L.apsm_model_packed_bytes(m2, 5, 300) == L.apsm_model_packed_bytes(32, 5, 300), m2
    assert L.apsm_model_packed_bytes(33, 6, 10) == 0          # invalid shape
    assert L.apsm_model_pack(None, None) == 1


_NEXT = [1 << 20]


def _addr(nbytes=1 << 20):
    """A distinct fake device address for each buffer (never dereferenced:
    these tests stop before any launch)."""
    a = _NEXT[0]
    _NEXT[0] += ((nbytes + (1 << 20) - 1) >> 20 << 20) + (1 << 20)
    return a


def _fresh_model(M2=32, K=6, cap=256, packed=True):
    return A._CModel(M2, K, cap, 0, _addr(M2 * cap * 4), _addr(cap * K * 4), _addr(K * M2 * 4), _addr(16),
                     _addr(1 << 22) if packed else None)


def _item(**kw):
    it = A._CBatchItem()
    it.model = kw.pop("model", None) or _fresh_model()
    base = dict(sigma2=0.5, P=64, rx_pilot=_addr(), sym_pilot=_addr(), S=100, modulation=2, rx=_addr(),
                soft=_addr(), hard=_addr(), truth=_addr(), err_count=_addr())
    base.update(kw)
    for k, v in base.items():
        setattr(it, k, v)
    return it


@needs_lib
def test_batch_create_plans_on_the_host():
    """apsm_batch_create validates and plans without touching the device; the
    workspace holds the job tables, one work item per 64 received vectors of
    the detectors on the split-FP16 path, and the claim counters."""
    L = A.library()
    items = (A._CBatchItem * 3)(_item(), _item(model=_fresh_model(M2=16, K=2, cap=100), S=65),
                                _item(model=_fresh_model(M2=128, K=16, cap=100), S=1000))
    h = ctypes.c_void_p()
    assert L.apsm_batch_create(ctypes.byref(_params()), items, 3, ctypes.byref(h)) == 0
    nbytes = L.apsm_batch_workspace_bytes(h)
    # 3 training jobs, 2 packing jobs, 2 detection jobs, 2 + 2 tiles, counters; each table 256-aligned
    assert nbytes >= 256 * 5 and nbytes % 256 == 0
    assert L.apsm_batch_train(h, None) == 1          # not bound to a workspace yet
    assert L.apsm_batch_detect(h, None) == 1
    assert L.apsm_batch_bind(h, None, nbytes, None) == A.ERR_WORKSPACE
    assert L.apsm_batch_bind(h, 256, nbytes - 1, None) == A.ERR_WORKSPACE   # too small
    assert L.apsm_batch_bind(h, 257, nbytes, None) == A.ERR_WORKSPACE       # misaligned
    assert L.apsm_batch_bind(None, 256, nbytes, None) == A.ERR_INVALID_ARG
    L.apsm_batch_destroy(h)
    L.apsm_batch_destroy(None)


BAD_ITEMS = [
    dict(sigma2=0.0), dict(P=0), dict(rx_pilot=None), dict(S=-1), dict(modulation=3),
    dict(truth=None), dict(soft=None, hard=None, err_count=None, truth=None), dict(rx=None),
    dict(model=_fresh_model(cap=8)),                     # capacity below the window
    dict(model=_fresh_model(packed=False)),              # packed form required for this shape
    dict(modulation=0),                                  # decisions asked without a modulation
]


@needs_lib
@pytest.mark.parametrize("kw", BAD_ITEMS)
def test_batch_create_rejects_bad_items(kw):
    L = A.library()
    items = (A._CBatchItem * 2)(_item(), _item(**kw))
    h = ctypes.c_void_p(1234)
    assert L.apsm_batch_create(ctypes.byref(_params()), items, 2, ctypes.byref(h)) != 0
    assert not h.value


def _overlapping(kind):
    """Two items whose buffers overlap in the way `kind` names."""
    a, b = _item(), _item()
    if kind == "soft_soft":           # two detectors writing the same outputs
        b.soft = a.soft
    elif kind == "soft_into_hard":    # one output running into another of the same item
        a.hard = a.soft + 100 * 6 * 2 * 4 - 8
    elif kind == "model_shared":      # two detectors training into one dictionary
        b.model.dict = a.model.dict + 64
    elif kind == "err_shared":
        b.err_count = a.err_count
    elif kind == "rx_is_output":      # received vectors of one item are another's soft outputs
        b.rx = a.soft
    elif kind == "pilots_in_alpha":
        b.rx_pilot = a.model.alpha + 4
    return a, b


@needs_lib
@pytest.mark.parametrize("kind", ["soft_soft", "soft_into_hard", "model_shared", "err_shared", "rx_is_output",
                                  "pilots_in_alpha"])
def test_batch_create_rejects_overlapping_buffers(kind):
    L = A.library()
    items = (A._CBatchItem * 2)(*_overlapping(kind))
    h = ctypes.c_void_p(1234)
    assert L.apsm_batch_create(ctypes.byref(_params()), items, 2, ctypes.byref(h)) == A.ERR_INVALID_ARG
    assert not h.value


@needs_lib
def test_batch_create_accepts_shared_inputs_and_adjacent_outputs():
    """Buffers that are only read may be shared; written buffers may touch
    (end of one = start of the next) without overlapping."""
    L = A.library()
    a, b = _item(), _item()
    b.rx, b.truth, b.rx_pilot, b.sym_pilot = a.rx, a.truth, a.rx_pilot, a.sym_pilot
    b.soft = a.soft + 100 * 6 * 2 * 4                # right after a's soft outputs
    b.err_count = a.err_count + 6 * 8
    items = (A._CBatchItem * 2)(a, b)
    h = ctypes.c_void_p()
    assert L.apsm_batch_create(ctypes.byref(_params()), items, 2, ctypes.byref(h)) == 0
    L.apsm_batch_destroy(h)
    # a detector with nothing to detect writes no outputs: its output pointers may alias
    c, d = _item(), _item(S=0)
    d.soft, d.hard, d.err_count = c.soft, c.hard, c.err_count
    items = (A._CBatchItem * 2)(c, d)
    assert L.apsm_batch_create(ctypes.byref(_params()), items, 2, ctypes.byref(h)) == 0
    L.apsm_batch_destroy(h)


@needs_lib
def test_batch_create_rejects_bad_arguments():
    L = A.library()
    items = (A._CBatchItem * 1)(_item())
    h = ctypes.c_void_p()
    assert L.apsm_batch_create(None, items, 1, ctypes.byref(h)) == 1
    assert L.apsm_batch_create(ctypes.byref(_params()), None, 1, ctypes.byref(h)) == 1
    assert L.apsm_batch_create(ctypes.byref(_params()), items, 0, ctypes.byref(h)) == 1
    assert L.apsm_batch_create(ctypes.byref(_params(mu=3.0)), items, 1, ctypes.byref(h)) == 1
    # sigma2 and dict_cap of the shared parameters are not used by batches
    assert L.apsm_batch_create(ctypes.byref(_params(sigma2=0.0, dict_cap=0)), items, 1, ctypes.byref(h)) == 0
    L.apsm_batch_destroy(h)


def _unr(**kw):
    base = dict(n_inst=2, P=16, M2=8, K=3, S=10, passes=4, ckpt_every=2, window=8, w_lin=0.5, w_gauss=0.5)
    base.update(kw)
    return A._CUnrolled(**base)


@needs_lib
def test_unrolled_workspace_and_validation():
    L = A.library()
    u = _unr()
    nbytes = L.apsm_unrolled_workspace_bytes(ctypes.byref(u))
    T = 32
    assert nbytes >= 2 * (2 * T * T * 4) and nbytes % 256 == 0
    # more passes per checkpoint segment -> a longer record
    assert L.apsm_unrolled_workspace_bytes(ctypes.byref(_unr(ckpt_every=4))) > nbytes
    for bad in (dict(n_inst=0), dict(P=0), dict(P=4096), dict(M2=7), dict(M2=256), dict(K=0), dict(K=17),
                dict(S=0), dict(passes=0), dict(ckpt_every=0), dict(window=0), dict(window=65),
                dict(w_lin=0.0, w_gauss=0.0), dict(w_lin=-1.0)):
        assert L.apsm_unrolled_workspace_bytes(ctypes.byref(_unr(**bad))) == 0, bad
    args = [1, 1, 1, 1, 1]
    assert L.apsm_unrolled_forward(ctypes.byref(_unr(K=0)), *args, 256, nbytes, 1, None) == 1
    assert L.apsm_unrolled_forward(ctypes.byref(u), *args, 256, nbytes - 1, 1, None) == A.ERR_WORKSPACE
    assert L.apsm_unrolled_forward(ctypes.byref(u), *args, 257, nbytes, 1, None) == A.ERR_WORKSPACE
    assert L.apsm_unrolled_forward(ctypes.byref(u), *args, None, nbytes, 1, None) == A.ERR_WORKSPACE
    assert L.apsm_unrolled_backward(ctypes.byref(u), *args, 256, nbytes - 1, None, 1, None) == A.ERR_WORKSPACE
    assert L.apsm_unrolled_forward(ctypes.byref(u), *args, 256, nbytes, None, None) == 1    # no loss
    assert L.apsm_unrolled_forward(ctypes.byref(u), None, 1, 1, 1, 1, 256, nbytes, 1, None) == 1
    assert L.apsm_unrolled_backward(ctypes.byref(u), *args, 256, nbytes, None, None, None) == 1


@needs_lib
def test_tune_cache_save_and_load(tmp_path):
    """The tuning cache round-trips through its JSON file; a malformed file
    or an unknown choice is rejected without merging anything."""
    import json
    A.shutdown()
    empty = tmp_path / "empty.json"
    A.tune_save(str(empty))
    assert json.loads(empty.read_text()) == {}
    entries = {"gfx950|hip70000000|detect|m2p32|k6": "wide", "gfx950|hip70000000|detect|m2p16|k4": "f16",
               "gfx950|hip70000000|form|00000000deadbeef": "persistent"}
    src = tmp_path / "cache.json"
    src.write_text(json.dumps(entries, indent=1))
    A.tune_load(str(src))
    out = tmp_path / "out.json"
    A.tune_save(str(out))
    assert json.loads(out.read_text()) == entries
    for bad in ('{"a": "fastest"}', '{"a": "wide"', "not json", '{"a" "wide"}'):
        f = tmp_path / "bad.json"
        f.write_text(bad)
        with pytest.raises(A.APSMError):
            A.tune_load(str(f))
    A.tune_save(str(out))
    assert json.loads(out.read_text()) == entries          # nothing merged from the bad files
    with pytest.raises(A.APSMError):
        A.tune_load(str(tmp_path / "missing.json"))
    A.shutdown()                                            # releases the cache
    A.tune_save(str(out))
    assert json.loads(out.read_text()) == {}


@needs_lib
def test_weights_modes_and_init_validation():
    """Violation weights exclude position weights; batches and the
    allocation-free entry point do not continue models (their kernel rows
    cover the pilots only)."""
    L = A.library()
    w = (ctypes.c_float * 16)(*([1.0] * 16))
    pw = ctypes.cast(w, ctypes.POINTER(ctypes.c_float))
    m = _model()
    assert L.apsm_train(ctypes.byref(_params(weights=1, pos_weights=pw)), 32, 6, 64, 1, 1, ctypes.byref(m),
                        None) == A.ERR_INVALID_ARG
    assert L.apsm_train(ctypes.byref(_params(weights=2, pos_weights=pw)), 32, 6, 64, 1, 1, ctypes.byref(m),
                        None) == A.ERR_INVALID_ARG
    items = (A._CBatchItem * 1)(_item())
    h = ctypes.c_void_p()
    assert L.apsm_batch_create(ctypes.byref(_params(init=2)), items, 1, ctypes.byref(h)) == 3
    assert L.apsm_train_noalloc(ctypes.byref(_params(init=2)), 32, 6, 64, 1, 1, ctypes.byref(m), None) == 3
    assert L.apsm_batch_create(ctypes.byref(_params(init=1, weights=1)), items, 1, ctypes.byref(h)) == 0
    L.apsm_batch_destroy(h)
    # active-set weights with the extrapolated relaxation, position weights with it
    assert L.apsm_batch_create(ctypes.byref(_params(weights=2, extrapolate=1)), items, 1, ctypes.byref(h)) == 0
    L.apsm_batch_destroy(h)
    assert L.apsm_batch_create(ctypes.byref(_params(extrapolate=1, pos_weights=pw)), items, 1,
                               ctypes.byref(h)) == 0
    L.apsm_batch_destroy(h)


@needs_lib
def test_mmse_and_track_validation():
    L = A.library()
    assert L.apsm_linear_mmse(None, 0.1, 32, 6, 1, 1, None) == 1
    assert L.apsm_linear_mmse(1, -0.1, 32, 6, 1, 1, None) == 1
    assert L.apsm_linear_mmse(1, float("nan"), 32, 6, 1, 1, None) == 1
    assert L.apsm_linear_mmse(1, 0.1, 31, 6, 1, 1, None) == 2
    assert L.apsm_linear_mmse(1, 0.1, 256, 6, 1, 1, None) == 3
    assert L.apsm_linear_mmse(1, 0.1, 32, 17, 1, 1, None) == 3
    assert L.apsm_linear_mmse(1, 0.1, 32, 6, 0, 1, None) == 0          # nothing to do
    p, m = _params(), _model()
    assert L.apsm_track(ctypes.byref(p), ctypes.byref(m), 10, 1, 0, 1, None, None, None, None) == 1   # no modulation
    assert L.apsm_track(ctypes.byref(p), ctypes.byref(m), 10, 1, 2, None, None, None, None, None) == 1
    assert L.apsm_track(ctypes.byref(p), ctypes.byref(m), -1, 1, 2, 1, None, None, None, None) == 2
    assert L.apsm_track(ctypes.byref(p), ctypes.byref(m), 0, None, 2, None, None, None, None, None) == 0
    assert L.apsm_track(ctypes.byref(_params(dict_cap=300)), ctypes.byref(m), 10, 1, 2, 1, None, None, None,
                        None) == 2
    assert L.apsm_track(ctypes.byref(p), ctypes.byref(m), 10, 1, 2, 1, None, 1, None, None) == 1   # truth w/o count


# ------------------------------------------------ generic projection engine

def _al(x):
    return (x + 255) & ~255


@needs_lib
def test_ball_workspace_bytes():
    L = A.library()
    for M2, K, cap in ((32, 6, 1024), (128, 16, 8192), (2, 1, 1), (6, 3, 70)):
        want = _al(cap * M2 * 4) + _al(cap * K * 8) + _al(K * 4)
        assert L.apsm_ball_workspace_bytes(M2, K, cap) == want
    for bad in ((3, 1, 10), (0, 1, 10), (32, 0, 10), (32, 17, 10), (256, 1, 10), (32, 1, 0)):
        assert L.apsm_ball_workspace_bytes(*bad) == 0


@needs_lib
def test_project_ball_rejects_bad_args():
    L = A.library()
    m = _model(M2=32, K=6, cap=256)
    need = L.apsm_ball_workspace_bytes(32, 6, 256)
    ws = 1 << 20                          # an aligned stand-in address; nothing is launched

    def call(model=m, sigma2=0.5, wl=0.5, wg=0.5, radius=1.0, ws=ws, nb=need):
        return L.apsm_project_ball(ctypes.byref(model) if model is not None else None, sigma2, wl, wg, radius,
                                   ws, nb, None, None)

    assert call(model=None) == A.ERR_INVALID_ARG
    assert call(model=_model(M2=7)) == A.ERR_SHAPE
    assert call(sigma2=0.0) == A.ERR_INVALID_ARG
    assert call(wl=0.0, wg=0.0) == A.ERR_INVALID_ARG
    assert call(wl=-1.0) == A.ERR_INVALID_ARG
    assert call(radius=-1.0) == A.ERR_INVALID_ARG
    assert call(radius=float("nan")) == A.ERR_INVALID_ARG
    assert call(radius=float("inf")) == A.ERR_INVALID_ARG
    assert call(ws=None) == A.ERR_WORKSPACE
    assert call(nb=need - 1) == A.ERR_WORKSPACE
    assert call(ws=ws + 16) == A.ERR_WORKSPACE            # not 256-byte aligned


@needs_lib
def test_pocs_rejects_bad_args():
    L = A.library()
    m = _model(M2=32, K=6, cap=256)
    need = L.apsm_ball_workspace_bytes(32, 6, 256)
    ws = 1 << 20

    def call(p=None, M2=32, K=6, P=64, rx=1, sym=1, model=m, radius=1.0, cycles=2, ws=ws, nb=need):
        p = p if p is not None else _params()
        return L.apsm_pocs(ctypes.byref(p), M2, K, P, rx, sym, ctypes.byref(model), radius, cycles, ws, nb, None)

    assert call(cycles=0) == A.ERR_INVALID_ARG
    assert call(p=_params(w_lin=0.0, w_gauss=1.0), cycles=2) == A.ERR_INVALID_ARG   # continued cycles need wL > 0
    assert call(p=_params(mu=2.5)) == A.ERR_INVALID_ARG
    assert call(radius=-0.5) == A.ERR_INVALID_ARG
    assert call(nb=need - 256) == A.ERR_WORKSPACE
    assert call(rx=None) == A.ERR_INVALID_ARG
    assert call(P=0) == A.ERR_SHAPE
    assert call(model=_model(M2=32, K=6, cap=300)) == A.ERR_SHAPE        # capacity differs from params
    assert call(K=5) == A.ERR_SHAPE


@needs_lib
def test_set_types_only_where_supported():
    """Entry points that train on hyperslabs only reject set kinds."""
    L = A.library()
    p = _params(set_types=1 << 20)
    m = _model()
    assert L.apsm_train_noalloc(ctypes.byref(p), 32, 6, 64, 1, 1, ctypes.byref(m), None) == A.ERR_UNSUPPORTED
    assert L.apsm_track(ctypes.byref(p), ctypes.byref(m), 10, 1, 2, 1, None, None, None, None) == A.ERR_UNSUPPORTED
    item = A._CBatchItem(model=_model(), sigma2=0.5, P=64, rx_pilot=1, sym_pilot=1, S=0, modulation=0)
    h = ctypes.c_void_p()
    assert L.apsm_batch_create(ctypes.byref(p), ctypes.byref(item), 1, ctypes.byref(h)) == A.ERR_UNSUPPORTED
