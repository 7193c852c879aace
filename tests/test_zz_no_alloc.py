"""darts_batch_render_noalloc: the batched render for callers that cannot
allocate, with the scenes' parameter blocks, work units and unit counters in
the library's fixed device array.  Checked against darts_batch_render (the
same kernel with memory the batch object allocated) on two calls in a row,
the second with a smaller batch, to the batch tests' bar (agreement to 1e-6
of the largest cell: only the order of the floating-point additions
differs), and the size limit is refused with a clear error."""
import numpy as np
import pytest
import torch

from paper_2402_03106_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_03106_amd import darts
    darts.lib()
    return darts


def _items(D, n, seed, lo_log2, hi_log2, mode="darts"):
    ws = W.batched(n, seed=seed, lo_log2=lo_log2, hi_log2=hi_log2)
    out = []
    for w in ws:
        t = D.build_da_tables(w["scene"]["medium"], w["dims"]) if D.MODES[mode] & D.EDA_DIR else None
        out.append((w["scene"], w["params"], mode, t))
    return out


def _reference(D, items, plan):
    b = D.Batch(items, plan)
    hi, lo = b.empty()
    b.render(hi, lo)
    torch.cuda.synchronize()
    img = (hi.double() + lo.double()).cpu().numpy()
    b.close()
    return img


def _check(got, want, offsets):
    for i in range(len(offsets) - 1):
        g, e = got[offsets[i]:offsets[i + 1]], want[offsets[i]:offsets[i + 1]]
        scale = max(np.abs(e).max(), 1e-30)
        assert np.abs(g - e).max() / scale <= 1e-6, i


@pytest.mark.parametrize("plan", [{"order": "ids", "block_threads": 256, "waves_per_cu": 16, "unit_paths": 1024},
                                  {"order": "tiles", "block_threads": 64, "waves_per_cu": 8, "unit_paths": 256}],
                         ids=["ids", "tiles"])
def test_noalloc_matches_batch_render(D, plan):
    first = _items(D, 12, 0xA11C, 10, 15)
    second = _items(D, 5, 0xB22D, 9, 13)          # smaller: fewer scenes and paths
    for items in (first, second):
        want = _reference(D, items, plan)
        hi = torch.zeros(want.size, dtype=torch.float32, device="cuda")
        lo = torch.zeros_like(hi)
        offsets = D.batch_render_noalloc(items, hi, lo, plan)
        torch.cuda.synchronize()
        assert offsets[-1] == want.size
        _check((hi.double() + lo.double()).cpu().numpy(), want, offsets)


def test_noalloc_refuses_what_does_not_fit(D):
    items = _items(D, 2, 0xC33E, 10, 11)
    hi = torch.zeros(10, dtype=torch.float32, device="cuda")
    with pytest.raises(D.DartsError, match="buffers hold"):
        D.batch_render_noalloc(items, hi, torch.zeros_like(hi))
    n = sum(int(np.prod(D.image_shape(it[0]))) for it in items)
    hi = torch.zeros(n, dtype=torch.float32, device="cuda")
    # 64-path id units of 2^22 paths per scene: more units than the fixed array holds
    big = [(sc, dict(p, n_paths=1 << 22), m, t) for sc, p, m, t in items]
    with pytest.raises(D.DartsError, match="raise unit_paths"):
        D.batch_render_noalloc(big, hi, torch.zeros_like(hi),
                               {"order": "ids", "block_threads": 64, "waves_per_cu": 8, "unit_paths": 64})
