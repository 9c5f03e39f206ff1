"""The C ABI driven from C with host AddressSanitizer: `tests/c/abi_driver.c`
linked against the library's host-ASan build walks every entry point twice
(keys, tables, encryption, batched / plain / device-pointer bootstraps, every
schedule, autotuning, timing, each step alone, the allocation-free key switch,
a general f, serving with admission, the 54-bit ring, a split ring, error paths)
and cross-checks the paths.  Built by `python -m paper_2310_12441_amd.build --asan`;
skipped when that build is absent."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "paper_2310_12441_amd", "lib_asan", "abi_driver")


def test_abi_driver_under_host_asan():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(DRIVER):
        pytest.skip("host-ASan build absent (python -m paper_2310_12441_amd.build --asan)")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    res = subprocess.run([DRIVER], capture_output=True, text=True, timeout=600, env=env)
    print(res.stdout[-2000:])
    assert res.returncode == 0, res.stderr[-4000:]
    assert "every check passed" in res.stdout
    assert "AddressSanitizer" not in res.stderr
