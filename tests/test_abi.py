"""The C-ABI library loads on the CPU and exports every function include/amnerf.h declares."""
import ctypes
import os
import re

import paper_2310_01881_amd as am

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "amnerf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(amnerf_[a-z_0-9]+)\s*\(", src)))


def test_header_declarations_are_exported():
    names = declared_functions()
    assert len(names) >= 14
    lib = ctypes.CDLL(am.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(am.EXPORTS) == sorted(names)


def test_calls_that_need_no_device():
    assert am.amnerf_version() == 100
    assert am.amnerf_mlp_param_count(4, 64) == 14724
    assert am.amnerf_mlp_param_count(2, 32) == 2180
    assert am.amnerf_mlp_param_count(0, 64) == -1
    assert am.amnerf_mlp_packed_bytes(4, 64, am.AMNERF_BF16, 512) > 0
    try:
        am.amnerf_mlp_packed_bytes(4, 48, am.AMNERF_BF16, 512)
        raise AssertionError("hidden=48 accepted")
    except am.AmnerfError as e:
        assert e.code == am.AMNERF_EINVAL and "unsupported" in am.amnerf_last_error()


def test_fp8_block_size():
    # float8 leaf block: float32 biases (n_hidden * hidden + 16, padded to 16 bytes), 16 scale
    # slots, then 32H + (n_hidden - 1) H^2 + 16H one-byte codes
    for nh, H in ((1, 32), (2, 32), (4, 64), (8, 64)):
        per = ((nh * H + 16) * 4 + 15) // 16 * 16 + 64 + 32 * H + (nh - 1) * H * H + 16 * H
        assert am.amnerf_mlp_packed_bytes(nh, H, am.AMNERF_FP8, 512) == per * 512
    assert am.amnerf_mlp_packed_bytes(4, 64, am.AMNERF_FP8, 1) < am.amnerf_mlp_packed_bytes(4, 64, am.AMNERF_BF16, 1) // 2


def test_no_device_fails_loudly():
    """Without a GPU the library reports an error: there is no CPU fallback."""
    import pytest
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    try:
        am.Context(0)
        raise AssertionError("a context was created without a device")
    except am.AmnerfError as e:
        assert e.code == am.AMNERF_EDEVICE and am.amnerf_last_error()
