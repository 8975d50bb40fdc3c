"""The C-ABI library loads and exports every function include/foe.h declares (CPU only: no compute calls)."""
import ctypes
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "foe.h")
LIB = os.path.join(ROOT, "paper_1404_5344_amd", "_lib", "libfoe.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(foe_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("foe_create", "foe_solve", "foe_destroy", "foe_solve_from", "foe_eval_gradient", "foe_eval_energy",
                 "foe_eval_prox", "foe_step", "foe_status_str", "foe_last_error", "foe_abi_version"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        import paper_1404_5344_amd.build as b
        b.build()
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert set(declared_functions()) <= exported


def test_host_only_calls():
    import paper_1404_5344_amd as foe
    assert foe.lib.foe_abi_version() == 2 == foe.ABI_VERSION
    with open(os.path.join(ROOT, "include", "foe.h")) as fh:
        assert "#define FOE_ABI_VERSION 2" in fh.read()
    assert foe.status_str(foe.ELINESEARCH) == "FOE_ELINESEARCH"
    p = foe.default_params(64, 64)
    assert p.num_filters == 48 and p.ksize == 7 and p.max_iters == 300 and p.beta == 0.8 and p.newton_iters == 30
    # parameter validation happens before any device call
    h = ctypes.c_void_p()
    k = (ctypes.c_float * (48 * 49))()
    th = (ctypes.c_float * 48)()
    p.beta = 1.5
    st = foe.lib.foe_create(ctypes.byref(p), k, th, None, ctypes.byref(h))
    assert st == foe.EINVAL and b"beta" in foe.lib.foe_last_error()
    # the split-FP16 engine takes taps below 2^14 only (AUTO falls back to FP32 operands instead)
    p.beta = 0.8
    p.engine = foe.ENGINE_MFMA_SPLIT
    k[5] = 20000.0
    st = foe.lib.foe_create(ctypes.byref(p), k, th, None, ctypes.byref(h))
    assert st == foe.EINVAL and b"split-FP16" in foe.lib.foe_last_error()
    p.engine = 4
    st = foe.lib.foe_create(ctypes.byref(p), k, th, None, ctypes.byref(h))
    assert st == foe.EINVAL and b"bad engine" in foe.lib.foe_last_error()


def test_noalloc_rejects_oversized_images_before_any_device_call():
    import paper_1404_5344_amd as foe
    k = (ctypes.c_float * (48 * 49))()
    th = (ctypes.c_float * 48)()
    dummy = ctypes.c_void_p(0x1000)   # never dereferenced: the size check comes first
    # 2048 x 2048 needs 5 planes of 16 MiB: beyond the 24 MiB workspace
    p = foe.default_params(2048, 2048)
    st = foe.lib.foe_solve_noalloc(ctypes.byref(p), k, th, None, dummy, None, dummy, None, None)
    assert st == foe.EINVAL and b"workspace" in foe.lib.foe_last_error()
    # so do the unfused path and NULL images
    p = foe.default_params(64, 64, fusion=1)
    st = foe.lib.foe_solve_noalloc(ctypes.byref(p), k, th, None, dummy, None, dummy, None, None)
    assert st == foe.EINVAL and b"fused" in foe.lib.foe_last_error()
    p = foe.default_params(64, 64)
    assert foe.lib.foe_solve_noalloc(ctypes.byref(p), k, th, None, None, None, dummy, None, None) == foe.EINVAL


def test_real_sar_preset_params():
    """Sec. III-C: the real SAR image has L = 5 looks and is despeckled with lambda1 = 50, lambda2 = 0.15
    (the looks table would interpolate other values for L = 5)."""
    import paper_1404_5344_amd as foe
    p = foe.real_sar_params(128, 96)
    assert (p.height, p.width, p.looks) == (128, 96, 5)
    assert p.lambda1 == 50.0 and p.lambda2 == 0.15
    assert p.num_filters == 48 and p.beta == 0.8 and p.model == 0
    assert foe.lib.foe_real_sar_params(None) == foe.EINVAL
    assert foe.lib.foe_batch_latency(None, None) == foe.EINVAL
