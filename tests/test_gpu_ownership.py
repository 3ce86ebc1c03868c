"""The device memory the library itself holds (the one exception to
caller-owned memory): a plan's geometry tables and a batch's maps and
descriptors.  Their reported size is the per-angle and per-block
bookkeeping it should be, and creating and destroying plans and batches
returns the device's free memory to where it was (nothing leaks)."""
import gc

import pytest
import torch

from gpu_helpers import say
from paper_2005_13471_amd import inputs

pytestmark = pytest.mark.gpu


def _free():
    torch.cuda.synchronize()
    gc.collect()
    return torch.cuda.mem_get_info()[0]


def test_plan_and_batch_tables_are_small_and_released():
    from paper_2005_13471_amd import gramct as gct
    N, n, zeta = 512, 720, 1.0
    P = gct.Plan(N, inputs.angles(n), 730, zeta=zeta)
    bytes_plan = P.device_bytes()
    # per angle: Gram and footprint parameters, back-projection polynomials
    # (a few hundred bytes); plus the P/2 twiddles and 2K+1 taps
    per_angle = (bytes_plan - 1024 * 8 * 3) / n
    say("plan tables", bytes_plan, "bytes;", per_angle, "per angle")
    assert 0 < bytes_plan and per_angle < 4096
    B = gct.Batch([P, gct.Plan(128, inputs.angles(90), 184, zeta=0.5)])
    say("batch maps", B.device_bytes())
    # one int2 per transform block of each pass, two descriptors per slice
    assert 0 < B.device_bytes() < 64 * (N * N + 256 * 256)
    del B, P
    before = _free()
    for i in range(20):
        p = gct.Plan(N, inputs.angles(n) + 0.001 * i, 730, zeta=zeta)
        b = gct.Batch([p])
        del b, p
    after = _free()
    say("free before", before, "after", after)
    # nothing held back (allocation granularity aside)
    assert after >= before - (4 << 20)
