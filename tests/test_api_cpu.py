"""The C ABI on the CPU: the library loads, exports every symbol the header
declares, and rejects bad arguments before touching HIP (so these run
without a GPU).  Also checks that the product never reaches the oracle."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in ("gs_fluid.h", "gs_cnn.h", "gs_batch.h")]

lib_mod = pytest.importorskip("paper_1812_07977_amd._lib")


def _lib():
    try:
        return lib_mod.lib()
    except lib_mod.LibraryMissing as e:
        pytest.fail(str(e))


def _declared():
    names = set()
    for path in HEADERS:
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(gs_(?:fluid|cnn|batch)_\w+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_binding_signatures():
    names = [n for n, _, _ in lib_mod.SIGNATURES]
    assert sorted(names) == _declared()


def test_library_exports_every_declared_symbol():
    L = _lib()
    for name in _declared():
        assert hasattr(L, name), name


G_OK = dict(nx=8, ny=8, nz=8, dx=0.125, dy=0.125, dz=0.125, gamma=1.4, cfl=0.5, bc=0, dtype=0)


def _create(**over):
    a = dict(G_OK)
    a.update(over)
    h = ctypes.c_void_p()
    st = _lib().gs_fluid_create(a["nx"], a["ny"], a["nz"], a["dx"], a["dy"], a["dz"], a["gamma"],
                                a["cfl"], a["bc"], a["dtype"], None, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("over", [
    dict(nx=0), dict(ny=-1), dict(nz=0),
    dict(dx=0.0), dict(dy=-0.1), dict(dz=math.inf), dict(dx=math.nan),
    dict(gamma=1.0), dict(gamma=0.5), dict(gamma=math.nan),
    dict(cfl=0.0), dict(cfl=1.5), dict(cfl=math.nan),
    dict(bc=2), dict(bc=-1), dict(dtype=2), dict(dtype=-1),
    dict(nx=1 << 16, ny=1 << 16, nz=2),
    dict(nx=1 << 15, ny=(1 << 14) + 1, nz=1),  # a plane of more than 2^29 cells
    dict(nx=1 << 15, ny=1 << 14, nz=1),        # exactly 2^29: its last cell ends at byte 2^32
])
def test_create_rejects_bad_arguments(over):
    st, h = _create(**over)
    assert st == lib_mod.GS_ERR_ARG
    assert not h.value
    assert _lib().gs_fluid_last_error(None).decode()


def test_create_rejects_null_out():
    L = _lib()
    st = L.gs_fluid_create(8, 8, 8, 0.1, 0.1, 0.1, 1.4, 0.5, 0, 0, None, None)
    assert st == lib_mod.GS_ERR_ARG


def test_null_handle_calls_are_argument_errors():
    L = _lib()
    d = ctypes.c_double()
    n = ctypes.c_int()
    assert L.gs_fluid_dt(None, None, ctypes.byref(d)) == lib_mod.GS_ERR_ARG
    assert L.gs_fluid_dt_last(None, ctypes.byref(d)) == lib_mod.GS_ERR_ARG
    assert L.gs_fluid_step_dt(None, None, 0.1, ctypes.byref(d)) == lib_mod.GS_ERR_ARG
    assert L.gs_fluid_step(None, None, 0.1) == lib_mod.GS_ERR_ARG
    assert L.gs_fluid_advance(None, None, 1, 0.0, None) == lib_mod.GS_ERR_ARG
    tot = (ctypes.c_double * 5)()
    assert L.gs_fluid_totals(None, None, tot) == lib_mod.GS_ERR_ARG
    assert L.gs_fluid_sync(None) == lib_mod.GS_ERR_ARG
    assert L.gs_fluid_get_time(None, ctypes.byref(d)) == lib_mod.GS_ERR_ARG
    assert L.gs_fluid_set_time(None, 0.0) == lib_mod.GS_ERR_ARG
    assert L.gs_fluid_set_stream(None, None) == lib_mod.GS_ERR_ARG
    assert L.gs_fluid_set_launch(None, 0, 0) == lib_mod.GS_ERR_ARG
    assert L.gs_fluid_profile(None, 1) == lib_mod.GS_ERR_ARG
    assert L.gs_fluid_kernel_ms(None, 0, ctypes.byref(d), ctypes.byref(n)) == lib_mod.GS_ERR_ARG
    L.gs_fluid_destroy(None)
    assert L.gs_fluid_last_error(None) is not None


NA_OK = dict(G_OK, U=4096, nsteps=1, t0=0.0, t_end=0.0, dt_log=None, t_out=None, flags_out=None)


def _noalloc(**over):
    a = dict(NA_OK)
    a.update(over)
    return _lib().gs_fluid_advance_noalloc(
        a["nx"], a["ny"], a["nz"], a["dx"], a["dy"], a["dz"], a["gamma"], a["cfl"], a["bc"],
        a["dtype"], a["U"], a["nsteps"], a["t0"], a["t_end"], a["dt_log"], a["t_out"],
        a["flags_out"], None)


@pytest.mark.parametrize("over", [
    dict(nx=0), dict(dz=math.nan), dict(gamma=1.0), dict(cfl=1.5), dict(bc=2), dict(dtype=3),
    dict(U=None), dict(U=4097), dict(nsteps=-1), dict(t0=math.inf), dict(t_end=-1.0),
    dict(t_end=math.nan), dict(dt_log=4100), dict(t_out=4), dict(flags_out=2),
    # workspace above the 96 MiB array: FP64 and FP32 both need 40 B per cell
    dict(nx=160, ny=128, nz=123), dict(nx=160, ny=128, nz=123, dtype=1),
])
def test_noalloc_rejects_bad_arguments_before_any_hip_call(over):
    # the state pointer is a host integer that is never dereferenced: every
    # case must fail in validation
    assert _noalloc(**over) == lib_mod.GS_ERR_ARG
    assert _lib().gs_fluid_last_error(None).decode()


def test_noalloc_size_limit_is_the_stated_cell_count():
    # 2,516,582 cells fit the 96 MiB workspace at 40 B per cell; one more does not
    assert 2516582 * 40 <= 96 << 20 < 2516583 * 40
    st = _noalloc(nx=2516583, ny=1, nz=1)
    assert st == lib_mod.GS_ERR_ARG
    assert "too large" in _lib().gs_fluid_last_error(None).decode()


def test_noalloc_valid_call_without_gpu_is_a_hip_error():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert _noalloc(nx=2516582, ny=1, nz=1) == lib_mod.GS_ERR_HIP


@pytest.mark.parametrize("dtype", [0, 1])
def test_workspace_bytes(dtype):
    L = _lib()
    n = 10 * 20 * 30
    ws = L.gs_fluid_workspace_bytes(10, 20, 30, dtype)
    assert ws >= n * 5 * 8                  # U(1), and for FP32 its increment
    assert ws - n * 5 * 8 < 128 * 1024      # plus reduction partials
    assert L.gs_fluid_workspace_bytes(0, 1, 1, dtype) == -1
    assert L.gs_fluid_workspace_bytes(1, 1, 1, 7) == -1


@pytest.mark.parametrize("dtype", [0, 1])
def test_valid_create_without_gpu_is_a_hip_error(dtype):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, h = _create(dtype=dtype)
    assert st == lib_mod.GS_ERR_HIP
    assert not h.value


def test_product_code_never_reaches_the_oracle():
    pkg = os.path.join(ROOT, "paper_1812_07977_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\boracle\b|gs_oracle|ora_", text), f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c")):
            text = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_1812_07977_amd" not in text and "gs_fluid" not in text, f


def _batch_create(count=2, dims=((8, 8, 8), (4, 6, 5)), gamma=1.4, cfl=0.5, bc=0, dtype=0,
                  states=(256, 512)):
    """gs_batch_create with host arrays; the state 'pointers' are never
    dereferenced before the arguments pass validation."""
    L = _lib()
    d = (ctypes.c_int * (3 * max(len(dims), 1)))(*[v for t in dims for v in t])
    s = (ctypes.c_void_p * max(len(states), 1))(*states) if states is not None else None
    h = ctypes.c_void_p()
    st = L.gs_batch_create(count, d if dims is not None else None, gamma, cfl, bc, dtype,
                           s, None, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("over", [
    dict(count=0), dict(count=-3), dict(count=1 << 17),
    dict(dims=((0, 8, 8), (4, 6, 5))), dict(dims=((8, 8, 8), (4, -1, 5))),
    dict(states=(256, 0)), dict(states=(256, 520)),
    dict(gamma=1.0), dict(gamma=math.nan), dict(cfl=0.0), dict(cfl=1.01),
    dict(bc=3), dict(dtype=5),
    dict(dims=((8, 8, 8), ((1 << 15) - 14, 1 << 14, 1))),  # padded plane over 2^29 cells
    dict(dims=((8, 8, 8), ((1 << 15) - 15, 1 << 14, 1))),  # padded plane of exactly 2^29 cells
])
def test_batch_create_rejects_bad_arguments(over):
    st, h = _batch_create(**over)
    assert st == lib_mod.GS_ERR_ARG
    assert not h.value
    assert _lib().gs_batch_last_error(None).decode()


def test_batch_create_rejects_null_arrays():
    L = _lib()
    h = ctypes.c_void_p()
    s = (ctypes.c_void_p * 1)(256)
    d = (ctypes.c_int * 3)(8, 8, 8)
    assert L.gs_batch_create(1, None, 1.4, 0.5, 0, 0, s, None, ctypes.byref(h)) == lib_mod.GS_ERR_ARG
    assert L.gs_batch_create(1, d, 1.4, 0.5, 0, 0, None, None, ctypes.byref(h)) == lib_mod.GS_ERR_ARG
    assert L.gs_batch_create(1, d, 1.4, 0.5, 0, 0, s, None, None) == lib_mod.GS_ERR_ARG


def test_batch_null_handle_calls_are_argument_errors():
    L = _lib()
    i = ctypes.c_int()
    t = (ctypes.c_double * 4)()
    assert L.gs_batch_set_launch(None, 0, 0) == lib_mod.GS_ERR_ARG
    assert L.gs_batch_autotune(None, None, ctypes.byref(i), ctypes.byref(i),
                               ctypes.byref(i)) == lib_mod.GS_ERR_ARG
    assert L.gs_batch_advance(None, 1, 0.0, 1) == lib_mod.GS_ERR_ARG
    assert L.gs_batch_times(None, t) == lib_mod.GS_ERR_ARG
    assert L.gs_batch_sync(None) == lib_mod.GS_ERR_ARG
    L.gs_batch_destroy(None)
    assert L.gs_batch_last_error(None) is not None


def test_cnn_parameter_count():
    # W1 32x5x27 + b1 32, W2 32x32x27 + b2 32, W3 5x32x27 + b3 5
    assert _lib().gs_cnn_param_count() == 32 * 5 * 27 + 32 + 32 * 32 * 27 + 32 + 5 * 32 * 27 + 5


@pytest.mark.parametrize("args", [
    (0, 8, 8, 1, 1.4), (8, -1, 8, 1, 1.4), (8, 8, 0, 1, 1.4),
    (1 << 10, 1 << 10, 1 << 9, 1, 1.4),
    (8, 8, 8, 2, 1.4), (8, 8, 8, -1, 1.4),
    (8, 8, 8, 1, 1.0), (8, 8, 8, 1, math.inf),
])
def test_cnn_create_rejects_bad_arguments(args):
    L = _lib()
    h = ctypes.c_void_p()
    assert L.gs_cnn_create(*args, None, ctypes.byref(h)) == lib_mod.GS_ERR_ARG
    assert not h.value
    assert L.gs_cnn_last_error(None).decode()
    assert L.gs_cnn_create(8, 8, 8, 1, 1.4, None, None) == lib_mod.GS_ERR_ARG


def test_cnn_null_handle_calls_are_argument_errors():
    L = _lib()
    d = ctypes.c_double()
    i = ctypes.c_int()
    v = (ctypes.c_double * 5)()
    E = lib_mod.GS_ERR_ARG
    assert L.gs_cnn_set_params(None, None) == E
    assert L.gs_cnn_get_params(None, None) == E
    assert L.gs_cnn_set_norm(None, v, v, v) == E
    assert L.gs_cnn_set_features(None, 0, 0.0) == E
    assert L.gs_cnn_forward(None, None, None) == E
    assert L.gs_cnn_restrict(None, None, None) == E
    assert L.gs_cnn_make_target(None, None, None, None) == E
    assert L.gs_cnn_gradients(None, None, None, None, ctypes.byref(d)) == E
    assert L.gs_cnn_train_step(None, None, None, 1e-3, ctypes.byref(d)) == E
    assert L.gs_cnn_correct(None, None) == E
    assert L.gs_cnn_counts(None, ctypes.byref(i), ctypes.byref(i)) == E
    assert L.gs_cnn_set_stream(None, None) == E
    L.gs_cnn_destroy(None)
    assert L.gs_cnn_last_error(None) is not None


@pytest.mark.parametrize("case", ["a_null", "c_null", "a_misaligned", "b_misaligned", "n_odd",
                                  "n_zero", "flags"])
def test_stream_probe_rejects_bad_arguments(case):
    # every case fails validation before a launch, so the fake (aligned,
    # never dereferenced) pointers are safe on any machine
    L = _lib()
    a, b, c = ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20), ctypes.c_void_p(3 << 20)
    n, flags = 1024, 0
    if case == "a_null":
        a = None
    elif case == "c_null":
        c = None
    elif case == "a_misaligned":
        a = ctypes.c_void_p((1 << 20) + 8)
    elif case == "b_misaligned":
        b = ctypes.c_void_p((2 << 20) + 8)
    elif case == "n_odd":
        n = 1023
    elif case == "n_zero":
        n = 0
    else:
        flags = 2
    assert L.gs_fluid_stream_probe(a, b, c, n, flags, None) == lib_mod.GS_ERR_ARG
    assert L.gs_fluid_last_error(None).decode()
