"""The persistent batched rollout's item loop must stay wave-uniform in the
generated gfx950 code (CPU only: compiles the kernel to assembly).

A divergent form of that loop (exits taken through EXEC masking) lets lanes
1..63 re-read a stale work ticket while lane 0 is masked off, which never
ends.  This guards the kernel source against changes that let the compiler
produce that form again."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1506_02869_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None,
                    reason="hipcc not available")
def test_batched_rollout_item_loop_is_uniform(tmp_path):
    out = tmp_path / "k.s"
    cmd = [HIPCC, "-x", "hip", "-O3", "-std=c++17", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "--cuda-device-only", "-S",
           os.path.join(CSRC, "kernels_rollout_batch.hip"), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    asm = out.read_text()
    names = re.findall(r"^(_ZN3smc18k_rollout_wm_batch\w+):", asm, re.M)
    assert len(names) == 16
    for n in names:
        start = asm.index(n + ":")
        body = asm[start:asm.index(".Lfunc_end", start)]
        # one returning atomic (the item fetch), executed by the whole wave
        fetch = [l for l in body.splitlines() if "global_atomic_add " in l and "sc0" in l]
        assert len(fetch) == 1, n
        assert "s_andn2_b64 exec, exec" not in body, f"{n}: divergent loop exit"
