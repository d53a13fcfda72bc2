"""apx_blend_noalloc (the entry point that allocates nothing) against apx_blend.

Both run the same kernels in the same order, so every output must agree bit for bit.
Two calls in a row, the second on a smaller input, check that the shared static
partial-sum array carries nothing from one call to the next; a size beyond the array's
limit must be refused before any device work.
"""

import math

import pytest
import torch

from paper_2411_03002_amd import binding as B

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    g = torch.Generator().manual_seed(seed)
    w = torch.where(torch.rand(n, generator=g, dtype=torch.float64) < 0.4, 0.0,
                    torch.rand(n, generator=g, dtype=torch.float64))
    e_eam = -3.0 + 0.1 * torch.randn(n, generator=g, dtype=torch.float64)
    e_ace = -3.0 + 0.1 * torch.randn(n, generator=g, dtype=torch.float64)
    f_eam = torch.randn(3, n, generator=g, dtype=torch.float64)
    f_ace = torch.randn(3, n, generator=g, dtype=torch.float64)
    return [t.cuda() for t in (w, e_eam, e_ace, f_eam, f_ace)]


def test_blend_noalloc_matches_blend():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2411_03002_amd import ops
    ctx = ops.Context(0)
    for n, seed in ((1_000_003, 5), (70_001, 6)):
        print(f"blend noalloc n={n} seed={seed}", flush=True)
        args = _inputs(n, seed)
        ref = ops.blend(ctx, *args)
        out = ops.blend(ctx, *args, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(out["e_site"], ref["e_site"])
        assert torch.equal(out["f"], ref["f"])
        assert torch.equal(out["e_pot"], ref["e_pot"])
        # the energy sum against an exactly rounded sum of the same site energies
        exact = math.fsum(ref["e_site"].cpu().tolist())
        assert abs(out["e_pot"].item() - exact) < 1e-9 * n
    # empty input: the sum is 0
    args = [t[..., :0].contiguous() for t in _inputs(4, 7)]
    out = ops.blend(ctx, *args, noalloc=True)
    torch.cuda.synchronize()
    assert out["e_pot"].item() == 0.0
    # beyond the static array's limit: refused on the host, no device work
    w, e_eam, e_ace, f_eam, f_ace = _inputs(8, 8)
    e_pot = torch.empty(1, dtype=torch.float64, device="cuda")
    P = lambda t: t.data_ptr()  # noqa: E731
    code = ctx.lib.apx_blend_noalloc(ctx.h, 65536 * 2048 + 1, P(w), P(e_eam), P(e_ace), P(f_eam), P(f_ace),
                                     P(e_eam), P(f_eam), P(e_pot))
    assert code == B.APX_EINVAL
    assert b"exceeds" in ctx.lib.apx_last_error(ctx.h)
    ctx.close()
