"""The FP32 hoisted adjoint must keep its step loops free of scratch memory
and its registers within three waves per SIMD (CPU only: compiles the kernel
to gfx950 assembly and reads the kernel descriptors).

The kernel's speed rests on the per-lane tapes, checkpoints and corner
caches staying in registers (168 VGPRs, three waves per SIMD) and on the
group index staying wave-uniform; this guards the source against changes
that push any of them into scratch memory or vector registers."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1506_02869_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _meta(asm, name, key):
    i = asm.index(".name:           " + name)
    block = asm[asm.rindex("- .", 0, i):asm.index("\n  - ", i) if "\n  - " in asm[i:] else len(asm)]
    return int(re.search(r"\." + key + r":\s+(\d+)", block).group(1))


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None,
                    reason="hipcc not available")
def test_hoisted_adjoint_fp32_registers(tmp_path):
    out = tmp_path / "g.s"
    cmd = [HIPCC, "-x", "hip", "-O3", "-std=c++17", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=on",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "--cuda-device-only", "-S",
           os.path.join(CSRC, "kernels_grad.hip"), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    asm = out.read_text()
    for mp in (32, 64, 128):
        name = f"_ZN3smc20k_rollout_grad_splitIfLi{mp}EEEvNS_10GradParamsEPKT_S4_PKdPKiS6_S6_PKaPd"
        assert _meta(asm, name, "vgpr_count") <= 168, mp
        # a few values spill around the block loop at most, never a tape
        assert _meta(asm, name, "private_segment_fixed_size") <= 32, mp
        start = asm.index(name + ":")
        body = asm[start:asm.index(".Lfunc_end", start)]
        # the block loop: from its header label to the last branch back to it
        hdr = re.search(r"^(\.LBB\w+):\s+; =>This Loop Header: Depth=1", body, re.M)
        assert hdr, mp
        label = hdr.group(1)
        back = max(m.start() for m in re.finditer(r"s_c?branch\w*\s+" + re.escape(label) + r"\b", body))
        assert "scratch_" not in body[hdr.start():back], mp
