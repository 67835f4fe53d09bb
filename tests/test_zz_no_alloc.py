"""The allocation-free event-driven CSR product (static device scratch)
against the workspace entry point and the oracle, through the C ABI: two
calls in a row on one GPU, the second with a smaller input; homogeneous
weights bit-exact (integer counts), heterogeneous data within 1e-5 of the sum
of |terms|."""
import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S

pytestmark = pytest.mark.gpu

dev = "cuda"


def _case(bp, seed, n_pre, n_post, p, frac, hetero, tile_index):
    K = O.max_gap(p)
    ip, ix = bp.csr_build(bp.JitConn(n_pre, n_post, K=K, seed=seed))
    nnz = int(ix.numel())
    data = torch.from_numpy(S.hetero_data(nnz, seed)).to(dev) if hetero else None
    e = S.events(n_pre, frac, seed)
    ev = torch.from_numpy(e).to(dev)
    tw = 0
    tp = None
    if tile_index:
        tw = -(-n_post // 8)
        tp = bp.csr_tile_index(ip, ix, n_post, tw)
    return ip, ix, data, ev, e, tp, tw


def _check(bp, seed, n_pre, n_post, p, frac, hetero, tile_index):
    ip, ix, data, ev, e, tp, tw = _case(bp, seed, n_pre, n_post, p, frac, hetero, tile_index)
    w = 0.0 if hetero else 0.6
    y_ws = bp.event_csr_matvec(ip, ix, data, w, n_post, ev, tp, tw)
    y_na = torch.full((n_post,), float("nan"), dtype=torch.float32, device=dev)
    bp.event_csr_matvec_noalloc(ip, ix, data, w, n_post, ev, y_na, tp, tw)
    torch.cuda.synchronize()
    a, b = y_na.cpu().numpy(), y_ws.cpu().numpy()
    ipn, ixn = ip.cpu().numpy(), ix.cpu().numpy()
    if not hetero:
        np.testing.assert_array_equal(a, b)
        cnt = O.event_csr_counts(ipn, ixn, n_post, e)
        np.testing.assert_array_equal(a, cnt.astype(np.float32) * np.float32(w))
    else:
        dn = data.cpu().numpy().astype(np.float64)
        ref = O.event_csr_matvec(ipn, ixn, dn, 0.0, n_post, e)
        scale = O.event_csr_matvec(ipn, ixn, np.abs(dn), 0.0, n_post, e)
        for y in (a, b):
            err = np.abs(y.astype(np.float64) - ref)
            assert np.all(err <= 1e-5 * scale + 1e-30)
            assert np.all(y[scale == 0] == 0.0)


@pytest.mark.parametrize("hetero", [False, True])
def test_noalloc_matches_workspace_entry_point_twice(hetero):
    import paper_2311_05106_amd as bp
    print(f"noalloc hetero={hetero}: 40000 x 60000 then 3000 x 5000", flush=True)
    # several tiles (tile index), several row chunks, ragged tail
    _check(bp, 31, 40_000, 60_000, 0.01, 0.1, hetero, True)
    # second call on the same GPU, smaller: one tile, the last call's
    # partials still in the array
    _check(bp, 32, 3_000, 5_000, 0.02, 0.3, hetero, False)


def test_noalloc_search_and_atomic_paths():
    import paper_2311_05106_amd as bp
    # sorted rows wider than a tile without an index (in-kernel search), then
    # an unsorted CSR (device-atomic accumulators in the static array)
    _check(bp, 33, 5_000, 40_000, 0.01, 0.2, False, False)
    n_pre, n_post = 2_000, 30_000
    rng = np.random.default_rng(5)
    rows = [np.sort(rng.choice(n_post, rng.integers(0, 40), replace=False))[::-1] for _ in range(n_pre)]
    ipn = np.concatenate([[0], np.cumsum([r.size for r in rows])]).astype(np.int32)
    ixn = np.concatenate(rows).astype(np.int32)
    e = S.events(n_pre, 0.3, 6)
    ip, ix, ev = (torch.from_numpy(x).to(dev) for x in (ipn, ixn, e))
    y_na = torch.empty(n_post, dtype=torch.float32, device=dev)
    bp.event_csr_matvec_noalloc(ip, ix, None, 0.5, n_post, ev, y_na, sorted_rows=False)
    cnt = O.event_csr_counts(ipn, ixn, n_post, e)
    np.testing.assert_array_equal(y_na.cpu().numpy(), cnt.astype(np.float32) * np.float32(0.5))
