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


@pytest.mark.parametrize("n", [2, 4098, 1 << 20, (1 << 20) + 2 * 517])
def test_hbm_probes_move_every_element(n):
    """The HBM probes touch every element exactly once: read sums integer data
    exactly, copy reproduces src, and the 3:1 kind writes the sum of the three
    source thirds; the byte count is 8n, 16n, 32n.  Sizes cover a single
    pair, a grid-stride remainder and whole rounds plus a ragged tail."""
    torch, _lib, _ = torch_mods()
    s = torch.cuda.current_stream().cuda_stream
    blocks = 16
    g = torch.Generator(device="cuda").manual_seed(5)
    src = torch.randint(-50, 50, (3 * n,), generator=g, device="cuda").to(torch.float64)
    dst = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    out = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    say(f"hbm probe n={n} read")
    st, by = _lib.ceiling_hbm(0, src.data_ptr(), 0, n, blocks, out.data_ptr(), s)
    assert st == 0 and by == 8 * n
    assert float(host(out).sum()) == float(host(src[:n]).sum())
    say(f"hbm probe n={n} copy")
    st, by = _lib.ceiling_hbm(1, src.data_ptr(), dst.data_ptr(), n, blocks, 0, s)
    assert st == 0 and by == 16 * n
    assert np.array_equal(host(dst), host(src[:n]))
    say(f"hbm probe n={n} three reads per write")
    st, by = _lib.ceiling_hbm(2, src.data_ptr(), dst.data_ptr(), n, blocks, 0, s)
    assert st == 0 and by == 32 * n
    h = host(src)
    assert np.array_equal(host(dst), h[:n] + h[n:2 * n] + h[2 * n:])
