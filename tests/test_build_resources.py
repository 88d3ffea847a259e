"""The built library's gfx950 kernels use no scratch memory.

Scratch (private segment) memory in these kernels means register spills or
locals the compiler could not keep in registers; in the entropy decoder's
symbol loop that costs several times its run time.  The check reads the
kernel descriptors of the code object that libjpt.so embeds, with the ROCm
LLVM tools (no GPU needed)."""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_2510_08166_amd import jpt

LLVM = "/opt/rocm/llvm/bin"
TOOLS = [os.path.join(LLVM, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf")]


def kernel_resources(so_path):
    """{kernel symbol: (private segment bytes, vgprs)} of the gfx950 code object in so_path."""
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    notes = ""
    with tempfile.TemporaryDirectory() as d:
        fat = os.path.join(d, "fat.bin")
        subprocess.run([TOOLS[0], "--dump-section", ".hip_fatbin=" + fat, so_path, os.path.join(d, "x.o")],
                       check=True, capture_output=True)
        data = open(fat, "rb").read()
        # one offload bundle per translation unit, concatenated (aligned)
        starts = [m.start() for m in re.finditer(re.escape(magic), data)]
        for i, a in enumerate(starts):
            part, co = os.path.join(d, "b%d.bin" % i), os.path.join(d, "b%d.co" % i)
            open(part, "wb").write(data[a:starts[i + 1] if i + 1 < len(starts) else len(data)])
            subprocess.run([TOOLS[1], "--unbundle", "--type=o", "--input=" + part,
                            "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", "--output=" + co], check=True,
                           capture_output=True)
            notes += subprocess.run([TOOLS[2], "--notes", co], check=True, capture_output=True, text=True).stdout
    out = {}
    # each kernel's metadata map lists its keys in order: .name, then
    # .private_segment_fixed_size, then (last of the three) .vgpr_count
    name = priv = None
    for line in notes.splitlines():
        m = re.match(r"\s+\.(name|private_segment_fixed_size|vgpr_count):\s+(\S+)", line)
        if not m:
            continue
        key, val = m.groups()
        if key == "name":
            name, priv = val, None
        elif key == "private_segment_fixed_size":
            priv = int(val)
        elif name is not None and priv is not None:
            out[name] = (priv, int(val))
            name = priv = None
    return out


@pytest.mark.skipif(not all(os.path.exists(t) for t in TOOLS), reason="ROCm LLVM tools not installed")
def test_no_kernel_uses_scratch():
    if not os.path.exists(jpt.LIB_PATH):
        pytest.skip("libjpt.so not built")
    res = kernel_resources(jpt.LIB_PATH)
    assert any("k_entropy" in k for k in res), "no entropy kernel found in the code object"
    assert any("k_resolve" in k for k in res) and any("k_mark" in k for k in res)
    for k, (priv, vgpr) in sorted(res.items()):
        print("%-100s scratch %4d B  vgprs %3d" % (k[:100], priv, vgpr))
    spills = {k: p for k, (p, _) in res.items() if p}
    assert not spills, "kernels using scratch memory: %s" % spills
