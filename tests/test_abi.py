"""The C-ABI library loads, exports every symbol the headers declare, and
rejects invalid arguments on the host before any device work (CPU only)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
import paper_1506_02869_amd as smc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in ("smc_mpc.h", "smc_kernels.h", "smc_batch.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(smc_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = smc.lib()
    declared = _declared()
    assert len(declared) >= 18
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(smc._SIGS) >= declared
    assert smc.smc_version().startswith("smc-mpc-gfx950")


@pytest.mark.parametrize("field,value", [
    ("N", 0), ("N", 65), ("S", 0), ("L", 0), ("M", 0), ("K", 0), ("dt", 0.0),
    ("grid", (1, 4, 4)), ("precision", 7), ("move", 9), ("wind_ell", 0.0),
    ("time_norm", -1.0),
])
def test_invalid_scenarios_rejected_on_host(field, value):
    s = synth.c1()
    if field == "N":
        # keep arrays consistent with N so that only the range check fires
        n = max(value, 1)
        s.update(N=n, kind=np.ones(n, np.int8), aircraft=np.tile(s["aircraft"][:1], (n, 1)),
                 targets=np.tile(s["targets"][:1], (n, 1)))
        sc, keep = smc.make_scenario_struct(s)
        sc.n_aircraft = value
    else:
        s[field] = np.array(value, dtype=np.int32) if field == "grid" else value
        sc, keep = smc.make_scenario_struct(s)
    h = C.c_void_p()
    st = smc.lib().smc_mpc_init(C.byref(sc), C.byref(h))
    assert st == smc.SMC_EINVAL
    assert h.value is None
    assert smc.lib().smc_last_error(None)


def test_bad_kind_and_null_arguments():
    s = synth.c1()
    s["kind"] = np.array([0, 3], np.int8)
    sc, keep = smc.make_scenario_struct(s)
    h = C.c_void_p()
    assert smc.lib().smc_mpc_init(C.byref(sc), C.byref(h)) == smc.SMC_EINVAL
    assert smc.lib().smc_mpc_init(None, C.byref(h)) == smc.SMC_EINVAL
    assert smc.lib().smc_mpc_step(None, 0, None, None, None, 1, None, None, None) == smc.SMC_EINVAL
    assert smc.lib().smc_k_philox(0, 0, 0, 1, 0, 0, -1, None, None) == smc.SMC_EINVAL
    smc.lib().smc_destroy(None)


def test_valid_scenario_without_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    sc, keep = smc.make_scenario_struct(synth.c1())
    h = C.c_void_p()
    st = smc.lib().smc_mpc_init(C.byref(sc), C.byref(h))
    assert st in (smc.SMC_EDEVICE, smc.SMC_ENOMEM)
    assert h.value is None


@pytest.mark.parametrize("cname,pyname", [
    ("smc_scenario", "Scenario"), ("smc_step_info", "StepInfo"),
    ("smc_batch_tuning", "BatchTuning"), ("smc_batch_info", "BatchInfo"),
])
def test_struct_layouts_match_the_headers(tmp_path, cname, pyname):
    """The binding's ctypes mirrors have the C structs' size and field offsets
    (the headers compiled by the host C compiler)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    py = getattr(smc, pyname)
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "smc_batch.h"',
             "int main(void) {", f'  printf("size %zu\\n", sizeof({cname}));']
    for f, _ in py._fields_:
        lines.append(f'  printf("{f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    assert int(out["size"]) == C.sizeof(py)
    for f, _ in py._fields_:
        assert int(out[f]) == getattr(py, f).offset, f
