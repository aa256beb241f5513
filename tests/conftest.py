import os
import shutil
import subprocess
import sys
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

XCHECK = os.path.join(ROOT, "tests", "xcheck")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU statistical test")


@pytest.fixture(scope="session")
def xcheck_dir():
    d = tempfile.mkdtemp(prefix="hyperim_xcheck_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def _torch_include():
    import torch.utils.cpp_extension as ce
    return ce.include_paths()[0]


@pytest.fixture(scope="session")
def torch_philox(xcheck_dir):
    """Path of PyTorch's Philox engine compiled as a filter program."""
    exe = os.path.join(xcheck_dir, "torch_px")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", _torch_include(),
                           os.path.join(XCHECK, "torch_px.cpp"), "-o", exe])
    return exe


@pytest.fixture(scope="session")
def rocrand_philox(xcheck_dir):
    """Path of rocRAND's Philox engine compiled (host side) as a filter program."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available for the rocRAND cross-check")
    exe = os.path.join(xcheck_dir, "roc_px")
    subprocess.check_call([hipcc, "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                           os.path.join(XCHECK, "roc_px.cpp"), "-o", exe],
                          stderr=subprocess.DEVNULL)
    return exe


def run_philox_filter(exe, ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    rec = np.concatenate([np.asarray(ctr, np.uint32).reshape(-1, 4),
                          np.asarray(key, np.uint32).reshape(-1, 2)], axis=1)
    out = subprocess.run([exe], input=np.ascontiguousarray(rec).tobytes(),
                         stdout=subprocess.PIPE, check=True).stdout
    return np.frombuffer(out, dtype=np.uint32).reshape(-1, 4)


def independent_coins(exe, seed, instance, pool, j, he, v, pos) -> np.ndarray:
    """Coins of channels computed with an independent Philox implementation:
    counter (j_lo, he, v, pool<<31 | j_hi<<24 | pos>>2), key (seed, instance),
    word pos & 3.  Arguments are equal-length integer arrays (or scalars)."""
    j = np.asarray(j, np.uint64)
    he, v, pos = (np.asarray(x, np.uint64) for x in (he, v, pos))
    n = max(x.size for x in (j, he, v, pos))
    j, he, v, pos = (np.broadcast_to(x, (n,)) for x in (j, he, v, pos))
    ctr = np.zeros((n, 4), np.uint64)
    ctr[:, 0] = j & 0xFFFFFFFF
    ctr[:, 1] = he
    ctr[:, 2] = v
    ctr[:, 3] = (np.uint64(pool) << np.uint64(31)) | ((j >> np.uint64(32)) << np.uint64(24)) | (pos >> np.uint64(2))
    key = np.zeros((n, 2), np.uint64)
    key[:, 0] = np.uint64(seed) & np.uint64(0xFFFFFFFF)
    key[:, 1] = instance
    out = run_philox_filter(exe, ctr.astype(np.uint32), key.astype(np.uint32))
    return out[np.arange(n), (pos & np.uint64(3)).astype(np.int64)]
