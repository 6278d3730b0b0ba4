"""CPU checks of the C ABI: the built library exports every declared entry point, the
ctypes structures match the C layout, and configuration validation fails loudly (these
paths return before any HIP call)."""
import ctypes
import os
import re
import subprocess

import pytest

import workloads as W
from paper_1910_01031_amd import abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "iewpf.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(iewpf_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = abi.load()
    declared = _declared()
    assert set(declared) == set(abi.EXPORTED)
    for name in declared:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", abi.LIB_PATH], capture_output=True,
                         text=True).stdout
    for name in declared:
        assert re.search(rf"\bT {name}\b", out), name


def test_struct_layouts_match_c(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include "iewpf.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(iewpf_config),'
                   ' sizeof(iewpf_obs), sizeof(iewpf_stats), offsetof(iewpf_config, seed),'
                   ' offsetof(iewpf_config, max_obs), offsetof(iewpf_stats, argmin_beta));'
                   ' return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert vals == [ctypes.sizeof(abi.IewpfConfig), ctypes.sizeof(abi.IewpfObs),
                    ctypes.sizeof(abi.IewpfStats), abi.IewpfConfig.seed.offset,
                    abi.IewpfConfig.max_obs.offset, abi.IewpfStats.argmin_beta.offset]


@pytest.mark.parametrize("kw,code", [
    (dict(nx=30), abi.IEWPF_E_SHAPE),               # not divisible by c_omega = 4
    (dict(nx=24, ny=24), abi.IEWPF_E_SHAPE),        # 6 coarse points < 7
    (dict(n_particles=0), abi.IEWPF_E_ARG),
    (dict(theta=0.5), abi.IEWPF_E_ARG),
    (dict(obs_sigma=0.0), abi.IEWPF_E_ARG),
    (dict(nx=17 * 8, ny=17 * 8, c_omega=17), abi.IEWPF_E_ARG),  # coarsening above 16
    (dict(n_particles=65536), abi.IEWPF_E_ARG),     # above the launch grids' y extent
    (dict(nx=16384, ny=10928), abi.IEWPF_E_SHAPE),  # 12 nx ny bytes >= 2^31 per particle
])
def test_invalid_configs_are_rejected(kw, code):
    lib = abi.load()
    cfg = W.tiny().replace(**kw)
    c = abi.make_config(cfg, 16)
    h = ctypes.c_void_p()
    rc = lib.iewpf_create(ctypes.byref(c), ctypes.byref(h))
    assert rc == code
    assert lib.iewpf_last_error().decode()
    assert not h.value


@pytest.mark.parametrize("value", ["0", "-3", "rows"])
def test_forced_strip_height_must_be_positive(value, monkeypatch):
    # the environment's strip height divides the grid height; non-positive values are
    # refused before any HIP call
    monkeypatch.setenv("IEWPF_SWE_STRIP", value)
    lib = abi.load()
    c = abi.make_config(W.tiny(), 16)
    h = ctypes.c_void_p()
    rc = lib.iewpf_create(ctypes.byref(c), ctypes.byref(h))
    assert rc == abi.IEWPF_E_ARG
    assert "IEWPF_SWE_STRIP" in lib.iewpf_last_error().decode()
    assert not h.value
