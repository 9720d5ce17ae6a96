"""The C-ABI library loads and exports every entry point include/mfwf.h declares (CPU only:
no compute call is made without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfwf.h")
LIB = os.path.join(ROOT, "paper_1210_4931_amd", "libmfwf.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mfwf_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1210_4931_amd import build
        build.build()
    from paper_1210_4931_amd import mfwf
    return mfwf.load()


def test_header_declares_the_boundary():
    names = declared()
    for n in ["mfwf_plan_create", "mfwf_plan_destroy", "mfwf_set_covariances", "mfwf_sht_inv",
              "mfwf_sht_fwd", "mfwf_fluctuation_rhs", "mfwf_solve", "mfwf_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (mfwf_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    for n in declared():
        assert getattr(lib, n) is not None


def test_binding_lists_every_export(lib):
    from paper_1210_4931_amd import mfwf
    assert sorted(mfwf.EXPORTED) == declared()


def test_last_error_and_destroy_null_without_gpu(lib):
    assert lib.mfwf_plan_destroy(None) == 0
    assert isinstance(lib.mfwf_last_error(), bytes)


def test_single_hip_runtime_in_process(lib):
    maps = open("/proc/self/maps").read()
    libs = {l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l}
    assert len(libs) == 1, libs


def test_no_kernel_uses_scratch_memory(lib):
    """Every kernel keeps its working set in registers and LDS: a stack object (scratch) in
    a hot loop turns register traffic into HBM traffic."""
    from paper_1210_4931_amd import build
    usage = build.resource_usage()
    kernels = {k: v for k, v in usage.items() if k.startswith("_ZN4mfwf")}
    assert kernels, "no resource report; build the library first"
    bad = {k: v.get("ScratchSize [bytes/lane]") for k, v in kernels.items()
           if v.get("ScratchSize [bytes/lane]", "0") != "0"}
    assert not bad, bad


def test_server_pool_bytes_is_host_only_and_validates(lib):
    from paper_1210_4931_amd.mfwf import MFWFError, Server
    b16 = Server.pool_bytes(16, 32, "f64", 2)
    assert b16 > 64 * 2**20  # fixed allowance for tables and workspaces
    assert Server.pool_bytes(512, 1024, "f64", 64) > Server.pool_bytes(512, 1024, "f64", 8)
    assert Server.pool_bytes(256, 512, "f32", 16) > Server.pool_bytes(128, 256, "f32", 16)
    assert Server.pool_bytes(2048, 4096, "f64", 1) > 4 * Server.pool_bytes(1024, 2048, "f64", 1)
    # the FP32 form at 2048 keeps lambda segment states (16 bytes per 16 table entries, about
    # 36 GB), not the FP32 table of about 140 GB
    assert 30e9 < Server.pool_bytes(2048, 4096, "f32", 1) < 100e9
    for args in [(24, 48, "f64", 2), (16, 65, "f64", 2), (16, 32, "f64", 0), (4096, 8192, "f64", 1),
                 (4096, 8192, "f32", 1), (2048, 4096, "f32", 0)]:
        with pytest.raises(MFWFError):
            Server.pool_bytes(*args)
