"""GPU parity at the full sizes of the two Gibbs workloads, in the launch
configuration the benchmark times: the trajectories of sampled chains equal
the oracle's, stored in tests/golden/config_chains.json by
tests/golden/make_config_chains.py (which calls only the oracle).

  * 18x18 annealing workload: 64 points x 4096 chains, geometric T 5.0 ->
    0.05 over 10^4 sweeps, autotuned tiling, one direct launch; chain k of
    point k for all 64 points.
  * uneven batch: 2048 instances, L in {6, 12, 18, 24, 36, 48}, 256 chains,
    5000 sweeps at fixed T, every size autotuned on its share of the batch,
    one hipGraph launch; one chain of each of 32 instances covering all six
    sizes.

Each chain's final spins and every 10th sweep's (M, B1, B2) must equal the
oracle's bit for bit.
"""
import hashlib
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
crbm = pytest.importorskip("paper_2511_20911_amd")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config_chains.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _pack(spins) -> str:
    bits = (np.asarray(spins).reshape(-1) > 0).astype(np.uint8)
    return np.packbits(bits, bitorder="little").tobytes().hex()


def _digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, "<i4").tobytes()).hexdigest()


def _check(smp, insts, recs, S, thin, launch_label):
    spins = torch.empty(smp.total_spins, dtype=torch.int8, device="cuda")
    tr = torch.empty((S // thin, smp.total_chains, 3), dtype=torch.int32, device="cuda")
    smp.sample(S, spins_out=spins, trace=tr, trace_every=thin)
    torch.cuda.synchronize()
    parts = smp.split_spins(spins)
    off = smp.chain_offsets
    cols = torch.tensor([int(off[r["instance"]]) + r["chain"] for r in recs], device="cuda")
    sub = tr.index_select(1, cols).cpu().numpy()
    del tr
    bad = []
    for q, r in enumerate(recs):
        k, ch = r["instance"], r["chain"]
        got = parts[k][ch].cpu().numpy()
        if _pack(got) != r["spins"]:
            bad.append((k, ch, "spins"))
        if _digest(sub[:, q, :]) != r[f"trace_every{thin}_sha256"]:
            bad.append((k, ch, "trace"))
    assert not bad, f"{launch_label}: {len(bad)} mismatches, first {bad[:8]}"


def test_anneal18_all_points_full_schedule_bit_exact():
    g = _golden()["anneal18"]
    S, thin, seed = g["sweeps"], g["thin"], g["seed"]
    assert len(g["chains"]) == 64 and sorted(r["instance"] for r in g["chains"]) == list(range(64))
    crbm.autotune(18, n_chains=8192, n_sweeps=40)
    J2S = (0.5, 1.0, 1.5, 2.0)
    insts = [crbm.Instance(L=18, J1=1.0, J2=J2S[k // 16], h=3.0 * (k % 16) / 15, n_chains=4096,
                           sched="geometric", T0=5.0, T1=0.05, id=k) for k in range(64)]
    smp = crbm.Sampler(insts, seed=seed, n_sweeps=S)
    _check(smp, insts, g["chains"], S, thin, f"18x18 anneal, tiling {crbm.get_tiling(18)}")


def test_uneven_batch_32_instances_all_sizes_bit_exact():
    from paper_2511_20911_amd import workloads
    g = _golden()["uneven"]
    S, thin, seed = g["sweeps"], g["thin"], g["seed"]
    pts = workloads.batched_uneven()
    assert {pts[r["instance"]].L for r in g["chains"]} == {6, 12, 18, 24, 36, 48}
    assert len(g["chains"]) == 32
    for r in g["chains"]:
        assert r["L"] == pts[r["instance"]].L
    for Lb in sorted({p.L for p in pts}):
        crbm.autotune(Lb, n_chains=sum(p.n_chains for p in pts if p.L == Lb), n_sweeps=20)
    insts = [crbm.Instance(L=p.L, J1=p.J1, J2=p.J2, h=p.h, n_chains=p.n_chains, sched=p.sched, T0=p.T0,
                           T1=p.T1, id=p.id) for p in pts]
    smp = crbm.Sampler(insts, seed=seed, n_sweeps=S, launch="graph")
    _check(smp, insts, g["chains"], S, thin, "uneven batch, graph launch")
