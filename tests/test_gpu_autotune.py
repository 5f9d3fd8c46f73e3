"""GPU: the autotuner of the batched launches (rw_batch_opts.autotune).

It times candidate launch shapes (paths per work item, i.e. chunk / 64 paths
per lane; waves per workgroup; wave occupancy of the persistent grid) on a
sample of the call's units and caches the fastest per shape key.  A launch
shape never changes a result: the tuned forward must give the untuned
forward's tallies bit for bit (exact integer sums) and the tuned adjoint the
untuned gradient to FP64 rounding.  With RW_AUTOTUNE_CACHE set, the choices
are written to that file and a new context reads them back instead of tuning
again."""
import os

import numpy as np
import pytest

from paper_2606_27604_amd import api, rw, workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from tests.gpu_common import ctx, geoms, media, np64  # noqa: E402


def _entries(path):
    out = {}
    with open(path) as f:
        for line in f:
            key, _, val = line.strip().partition("|")
            chunk, wpw, per_cu = (int(x) for x in val.split())
            out[key] = (chunk, wpw, per_cu)
    return out


def test_autotuned_calls_match_untuned_and_the_cache_round_trips(tmp_path, monkeypatch):
    cache = str(tmp_path / "tune.txt")
    monkeypatch.setenv("RW_AUTOTUNE_CACHE", cache)
    wl = workloads.config2(paths=1 << 16)
    sub = wl.subset(np.arange(24))
    m = media(sub.sigma_t, sub.albedo, sub.g, sub.weight)
    g, _ = geoms(3, sub.n_rel)
    N, n = sub.paths_per_unit, sub.n_units
    rng = np.random.default_rng(5)
    cR = torch.ones(n, dtype=torch.float32, device="cuda")
    cB = torch.from_numpy(rng.standard_normal((n, g.n_bins + 2)).astype(np.float32)).cuda()

    tuned = rw.Context(0)  # reads the (empty) cache at its first batched call
    mask_t = rw.new_path_mask(n, N)
    res_t = api.forward(tuned, m, g, N, 13, autotune=True, path_mask=mask_t)
    adj_t = api.adjoint(tuned, m, g, N, 13, cot_R=cR, cot_bins=cB, path_mask=mask_t)
    assert rw.rw_check(tuned, res_t.tally.flags) == 0 and rw.rw_check(tuned, adj_t[3]) == 0
    # the adjoint tuned too (same options as the forward's call)
    rw.rw_batch_adjoint(tuned, m, g, None, N, 13, cR, cB, adj_t[0], adj_t[1], adj_t[2], adj_t[3],
                        autotune=True, path_mask=mask_t)
    torch.cuda.synchronize()

    mask_u = rw.new_path_mask(n, N)
    res_u = api.forward(ctx(), m, g, N, 13, path_mask=mask_u)
    adj_u = api.adjoint(ctx(), m, g, N, 13, cot_R=cR, cot_bins=cB, path_mask=mask_u)
    torch.cuda.synchronize()
    assert torch.equal(res_t.tally.R, res_u.tally.R)
    assert torch.equal(res_t.tally.bins, res_u.tally.bins)
    assert torch.equal(res_t.tally.vertices, res_u.tally.vertices)
    assert torch.equal(mask_t, mask_u)
    G, Gu = np64(adj_t[0]), np64(adj_u[0])
    assert np.all(np.abs(G - Gu) <= 1e-9 * (np.abs(Gu) + np.abs(Gu).max(0))), np.abs(G - Gu).max()
    assert torch.equal(adj_t[2], adj_u[2])

    # the cache holds a forward and an adjoint entry with valid shapes
    ent = _entries(cache)
    fwd = [k for k in ent if " fwd " in k and k.endswith("m1")]
    adj = [k for k in ent if " adj " in k and k.endswith("m1")]
    assert fwd and adj, ent
    for chunk, wpw, per_cu in ent.values():
        assert chunk % 64 == 0 and 1024 <= chunk <= 8192 and wpw in (1, 2, 4) and per_cu >= 0
    stamp = os.stat(cache).st_mtime_ns
    text = open(cache).read()

    # a new context reads the cache and does not tune again (the file stays as it is)
    again = rw.Context(0)
    res_a = api.forward(again, m, g, N, 13, autotune=True, path_mask=rw.new_path_mask(n, N))
    torch.cuda.synchronize()
    assert torch.equal(res_a.tally.R, res_u.tally.R)
    assert os.stat(cache).st_mtime_ns == stamp and open(cache).read() == text

    # a cache line with an invalid shape is ignored (the call tunes that key again)
    with open(cache, "w") as f:
        for k in ent:
            f.write(f"{k}|100 3 0\n")
    bad = rw.Context(0)
    res_b = api.forward(bad, m, g, N, 13, autotune=True, path_mask=rw.new_path_mask(n, N))
    torch.cuda.synchronize()
    assert torch.equal(res_b.tally.R, res_u.tally.R)
    ent2 = _entries(cache)
    assert all(v[0] % 64 == 0 and v[1] in (1, 2, 4) for v in ent2.values())
