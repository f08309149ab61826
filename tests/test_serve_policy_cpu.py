"""The server's admission and batching policy, compiled and run on the CPU
(the header has no HIP dependency), and the server ABI's argument checks."""
import ctypes
import os
import subprocess

import pytest

from paper_1604_04815_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_policy_unit(tmp_path):
    exe = str(tmp_path / "serve_policy_test")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_1604_04815_amd", "csrc"),
                    os.path.join(ROOT, "tests", "serve_policy_test.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout


@pytest.fixture(scope="module")
def lib():
    return binding.load()


def test_server_config_validation(lib):
    cfg = binding.ServerConfig()
    assert lib.lscan_server_default_config(ctypes.byref(cfg)) == binding.OK
    assert cfg.num_streams == 2 and cfg.groups_per_cu == 0 and cfg.hbm_budget_bytes == 32 << 30
    h = ctypes.c_void_p()
    for field, value in (("num_streams", 0), ("groups_per_cu", -1), ("hbm_budget_bytes", 0), ("max_queue", 0),
                         ("max_batch", 0), ("num_streams", 4), ("groups_per_cu", 2)):
        bad = binding.ServerConfig()
        lib.lscan_server_default_config(ctypes.byref(bad))
        setattr(bad, field, value)
        assert lib.lscan_server_create(ctypes.byref(bad), ctypes.byref(h)) == binding.ERR_INVALID_ARG, field
    assert lib.lscan_server_create(None, ctypes.byref(h)) == binding.ERR_INVALID_ARG


def test_server_null_handles(lib):
    r = binding.Request()
    t = ctypes.c_uint64()
    res = binding.Result()
    assert lib.lscan_submit(None, ctypes.byref(r), ctypes.byref(t)) == binding.ERR_INVALID_ARG
    assert lib.lscan_poll(None, 1, ctypes.byref(res)) == binding.ERR_INVALID_ARG
    assert lib.lscan_wait(None, 1, ctypes.byref(res)) == binding.ERR_INVALID_ARG
    assert lib.lscan_server_destroy(None) == binding.ERR_INVALID_ARG
