"""GPU parity of rsrr_sample_batched (ragged batches of instances, size buckets,
device-side refinement, hipGraph capture and replay, autotuning of the panel width and
the update tile)
against the CPU oracle.  Bar: every block X_k within 1e-10 (relative
Frobenius) of the oracle's LAPACK solve, reported residuals <= 1e-10."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import rsrr_oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_07951_amd import rsrr
    rsrr.lib()
    return rsrr


def _items(R, sizes, N, L, seed=3000):
    items, hosts = [], []
    for i, n in enumerate(sizes):
        nep = W.rotated_diagonal_qep(int(n), seed + i)
        U = W.probes(int(n), L, seed + 100 + i)
        z, _ = O.ellipse(5j, 4.0, 1.0, N)
        items.append(R.BatchItem(R.DeviceNEP(nep), z, U))
        hosts.append((nep, z, U))
    return items, hosts


def _check(R, items, hosts, infos, tol=1e-10):
    torch.cuda.synchronize()
    for it, (nep, z, U), inf in zip(items, hosts, infos):
        prob = O.Problem(nep)
        S = R.from_colmajor(it.S, nep.n)
        L = U.shape[1]
        for k, zk in enumerate(z):
            Xo = O.solve_point(prob.T(zk), U)
            X = S[:, k * L:(k + 1) * L]
            assert np.linalg.norm(X - Xo) <= tol * np.linalg.norm(Xo), (nep.n, k)
            assert inf[k]["resid"] <= 1e-10
            # these points are well conditioned: the factorisation itself must be right
            # (a redo on the FP64 path would hide a wrong LU)
            assert inf[k]["fallback"] == 0 and inf[k]["info"] == 0, (nep.n, k, inf[k])


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_ragged_sizes(R, prec):
    ctx = R.rsrr_create(0)
    sizes = [5, 64, 65, 100, 130, 200, 63, 257]
    items, hosts = _items(R, sizes, N=6, L=4)
    infos, code = R.rsrr_sample_batched(ctx, items, prec=prec)
    _check(R, items, hosts, infos)
    ctx.close()


def test_batched_graph_replays_match_eager(R):
    ctx = R.rsrr_create(0)
    sizes = [70, 128, 129, 190]
    items, hosts = _items(R, sizes, N=8, L=3, seed=4000)
    infos, _ = R.rsrr_sample_batched(ctx, items, prec=1)
    eager = [it.S.clone() for it in items]
    _check(R, items, hosts, infos)
    for rep in range(4):
        for it in items:
            it.S.zero_()
        infos, _ = R.rsrr_sample_batched(ctx, items, prec=1, flags=R.RSRR_BATCH_GRAPH)
        torch.cuda.synchronize()
        # some eager work and a synchronisation between replays
        tmp = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        for it, e in zip(items, eager):
            assert torch.equal(it.S, e), f"replay {rep} differs from the eager result"
        assert all(i["resid"] <= 1e-10 for inf in infos for i in inf)
    ctx.close()


def test_batched_autotune_writes_cache(R, tmp_path, monkeypatch):
    """The autotuner times every (panel width, update tile) candidate on each bucket and caches the
    winner per (bucket, precision, arch) as JSON; a fresh context that reads the cache reproduces
    the tuned call's S bit for bit."""
    import json
    f = tmp_path / "tune.json"
    monkeypatch.setenv("RSRR_TUNE_FILE", str(f))
    ctx = R.rsrr_create(0)
    items, hosts = _items(R, [300, 310, 700], N=5, L=2, seed=5000)
    infos, _ = R.rsrr_sample_batched(ctx, items, prec=1, flags=R.RSRR_BATCH_AUTOTUNE)
    _check(R, items, hosts, infos)
    tuned = [it.S.clone() for it in items]
    ctx.close()
    doc = json.loads(f.read_text())
    assert doc["arch"].startswith("gfx9")
    ent = {(e["P"], e["prec"]): e for e in doc["entries"]}
    assert set(ent) == {(320, "c64"), (704, "c64")}
    for e in ent.values():
        assert e["nb"] in (32, 64, 128) and e["update_tile"] in (0, 1, 2, 3) and e["ms"] > 0
        assert e["update_tile_name"].endswith("4waves")
    ctx = R.rsrr_create(0)
    for it in items:
        it.S.zero_()
    R.rsrr_sample_batched(ctx, items, prec=1)
    torch.cuda.synchronize()
    for it, t in zip(items, tuned):
        assert torch.equal(it.S, t)
    ctx.close()


def test_batched_matches_single_instance_calls(R):
    """The same instance gives the same S alone and inside a mixed batch (bucket-independent kernels)."""
    ctx = R.rsrr_create(0)
    items, hosts = _items(R, [150, 160, 170], N=4, L=2, seed=6000)  # one size bucket (192)
    R.rsrr_sample_batched(ctx, items, prec=1)
    mixed = [it.S.clone() for it in items]
    for it in items:
        it.S.zero_()
        R.rsrr_sample_batched(ctx, [it], prec=1)
    torch.cuda.synchronize()
    for it, m in zip(items, mixed):
        assert torch.equal(it.S, m)
    ctx.close()


@pytest.mark.parametrize("tile", [0, 1, 2, 3])
@pytest.mark.parametrize("nb", [32, 64, 128])
def test_batched_every_panel_width(R, tmp_path, monkeypatch, nb, tile):
    """Each panel width and update tile the autotuner may pick, forced through the JSON cache, on
    buckets whose size is and is not a multiple of the width (P = 128, 192, 256, 320)."""
    import json
    f = tmp_path / "tune.json"
    entries = [{"P": P, "prec": "c64", "nb": nb, "update_tile": tile, "ms": 1.0} for P in (128, 192, 256, 320)]
    # the library's own layout: one entry per line
    f.write_text('{"arch": "gfx950", "entries": [\n' + ",\n".join(json.dumps(e) for e in entries) + "\n]}\n")
    json.loads(f.read_text())
    monkeypatch.setenv("RSRR_TUNE_FILE", str(f))
    ctx = R.rsrr_create(0)
    items, hosts = _items(R, [100, 150, 250, 300], N=4, L=3, seed=7000 + nb + 10 * tile)
    infos, code = R.rsrr_sample_batched(ctx, items, prec=1)
    assert code == R.RSRR_OK
    _check(R, items, hosts, infos)
    ctx.close()
