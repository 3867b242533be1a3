"""The FP64 ceiling probes (roofline support) through the C ABI: each launch
runs, reports the exact flop count of its loop (four MFMA chains per wave,
eight FMA chains per lane, 256 threads per workgroup) and stores finite
values."""
import numpy as np
import pytest

from tests.gpu_util import host, say, torch_mods

pytestmark = pytest.mark.gpu


def test_ceiling_probes_run_and_count():
    torch, _lib, _ = torch_mods()
    s = torch.cuda.current_stream().cuda_stream
    blocks = 8
    out = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    for kind, per_iter in ((0, 4 * 2048 * 4), (1, 256 * 8 * 2)):
        for iters in (1, 7):
            say(f"ceiling probe kind={kind} iters={iters}")
            st, fl = _lib.ceiling_fp64(kind, blocks, iters, out.data_ptr(), s)
            assert st == 0, st
            assert fl == blocks * iters * per_iter
            v = host(out)
            assert np.all(np.isfinite(v))
