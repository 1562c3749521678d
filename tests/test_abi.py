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
    assert am.amnerf_version() == 201
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


def test_struct_layouts_match_the_header(tmp_path):
    """Every C struct the binding mirrors has the header's size and field offsets (a C
    program compiled against include/amnerf.h prints them)."""
    import shutil
    import subprocess
    import pytest
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {name: getattr(am, name) for name in dir(am)
               if name.startswith("amnerf_") and isinstance(getattr(am, name), type)
               and issubclass(getattr(am, name), ctypes.Structure)}
    assert len(structs) >= 14
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "amnerf.h"', 'int main(void) {']
    for name, st in structs.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for f, _ in st._fields_:
            lines.append('  printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, f, name, f))
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                                check=True).stdout.splitlines())
    for name, st in structs.items():
        assert int(got[name + " size"]) == ctypes.sizeof(st), name
        for f, _ in st._fields_:
            assert int(got["%s.%s" % (name, f)]) == getattr(st, f).offset, (name, f)
