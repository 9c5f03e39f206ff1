"""The allocation-free key switch (mm_keyswitch_noalloc) against mm_keyswitch.

The entry point keeps its partial sums in a fixed device array per GPU; two
calls in a row, the second smaller, must each give the bits of the allocating
entry point on the same input (eq. equ-key-swi), and sizes beyond the array are
refused before anything runs.
"""
import numpy as np
import pytest

from synth import PRESETS, key_draws

pytestmark = pytest.mark.gpu
Q = 2147352577


def test_keyswitch_noalloc_matches_keyswitch_twice():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_12441_amd import binding as b
    p = PRESETS["paper_shaped"]["params"]
    ctx = b.Context(p, key_draws(p, 41))
    try:
        ctx.device_init(0)
        rng = np.random.default_rng(41)
        for count in (3000, 37):
            print("noalloc key switch, count", count, flush=True)
            lw = rng.integers(0, Q, (count, p.N + 1), dtype=np.uint32)
            want = ctx.keyswitch(lw)
            dev_in = torch.from_numpy(lw.view(np.int32)).cuda()
            dev_out = torch.full((count, p.n + 1), -1, dtype=torch.int32, device="cuda")
            ctx.keyswitch_noalloc(dev_in, dev_out)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(dev_out.cpu().numpy().view(np.uint32), want, err_msg=f"count {count}")
        # beyond the 64 MiB scratch: count * (n + 1) * 8 > 2^26 is refused before any launch
        big = (64 << 20) // ((p.n + 1) * 8) + 1
        dev_in = torch.zeros((big, p.N + 1), dtype=torch.int32, device="cuda")
        dev_out = torch.zeros((big, p.n + 1), dtype=torch.int32, device="cuda")
        with pytest.raises(b.MMError) as e:
            ctx.keyswitch_noalloc(dev_in, dev_out)
        assert e.value.code == b.MM_EINVAL
    finally:
        ctx.close()


def test_keyswitch_noalloc_needs_device_init():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_12441_amd import binding as b
    p = PRESETS["tiny"]["params"]
    ctx = b.Context(p, key_draws(p, 42))
    try:
        x = torch.zeros((1, p.N + 1), dtype=torch.int32, device="cuda")
        y = torch.zeros((1, p.n + 1), dtype=torch.int32, device="cuda")
        with pytest.raises(b.MMError) as e:
            ctx.keyswitch_noalloc(x, y)
        assert e.value.code == b.MM_ESTATE
    finally:
        ctx.close()
