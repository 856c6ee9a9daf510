"""Pass schedules (what the autotuner picks) on the GPU: every candidate schedule computes the same spectra
within the FP32 path's tolerance (Stokes, max_k |P - P_ref| / I_ref,k <= 1e-5 against the FP64 oracle), the
grouped launches honour per-instance schedules bit for bit, and the tuner records its choice in its JSON
cache and reads it back."""
import json
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1412_1256_amd as pk
    pk.lib()
    return torch, pk, torch.device("cuda:0")


@pytest.mark.parametrize("log2n,bits", [(14, 8), (16, 2), (18, 8)])
def test_every_candidate_matches_oracle(env, log2n, bits):
    torch, pk, dev = env
    F = 32 if log2n < 18 else 8
    inst = synth.make_correlated_noise(bits, 0.3, 1 << log2n, F, seed_extra=log2n)
    acc, nf, s2, _ = oracle.run_instance(inst)
    ref = oracle.stokes(acc, nf, s2)
    packed = torch.from_numpy(inst["packed"]).to(dev)
    cands = pk.schedule_candidates(pk.Instance.from_synth(inst))
    say(f"N=2^{log2n} bits={bits}: {len(cands)} schedules")
    for s in cands:
        plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev, schedules=[s])
        plan.reset()
        plan.accumulate(packed)
        got = plan.stokes().cpu().numpy().astype(np.float64)
        if F >= 32:
            e = np.max(np.abs(got - ref) / ref[:, 0:1, :])
        else:
            e = np.max(np.abs(got - ref)) / np.mean(ref[:, 0, :])
        say(f"  {s}: err {e:.2e}")
        assert e < 1e-5, s


# rows of 1024 and 2048 points are held as 16 points per lane (passes of radix 8, 8 or 16, and 16): splits that put
# 1024 or 2048 points in the row pass, through the plain, fused-Stokes and grouped row passes
@pytest.mark.parametrize("log2n,log2n1,bits,F", [(19, 9, 8, 8), (20, 10, 2, 4), (20, 9, 8, 4), (19, 8, 2, 8)])
def test_wide_rows_match_oracle(env, log2n, log2n1, bits, F):
    torch, pk, dev = env
    inst = synth.make_correlated_noise(bits, 0.3, 1 << log2n, F, seed_extra=log2n + 7)
    acc, nf, s2, _ = oracle.run_instance(inst)
    ref = oracle.stokes(acc, nf, s2)
    packed = torch.from_numpy(inst["packed"]).to(dev)
    say(f"N=2^{log2n} as 2^{log2n1} x 2^{log2n - log2n1}, bits={bits}, F={F}")
    for slots in (1, 2):
        plan = pk.Plan([pk.Instance.from_synth(inst)], device=dev,
                       schedules=[pk.Schedule(log2_n1=log2n1, rowpass_slots=slots)])
        plan.reset()
        got = plan.accumulate_stokes(packed)[0].cpu().numpy().astype(np.float64)
        e = np.max(np.abs(got - ref)) / np.mean(ref[:, 0, :])
        say(f"  slots={slots}: err {e:.2e}")
        assert e < 1e-5
    # two instances of this split in one grouped plan: the grouped row pass, bitwise as separate plans
    other = synth.make_correlated_noise(bits, 0.1, 1 << log2n, F, seed_extra=log2n + 8)
    p2 = torch.from_numpy(other["packed"]).to(dev)
    sch = pk.Schedule(log2_n1=log2n1)
    grp = pk.Plan([pk.Instance.from_synth(inst), pk.Instance.from_synth(other)], device=dev, schedules=[sch, sch])
    grp.reset()
    grp.accumulate([packed, p2])
    for i, (d, buf) in enumerate(((inst, packed), (other, p2))):
        one = pk.Plan([pk.Instance.from_synth(d)], device=dev, schedules=[sch])
        one.reset()
        one.accumulate(buf)
        assert torch.equal(grp.spectra(i)[0], one.spectra()[0]), i


def test_grouped_launches_honour_schedules(env):
    torch, pk, dev = env
    say("grouped plan with per-instance schedules")
    insts = [synth.make_correlated_noise(b, 0.2, 1 << e, F, seed_extra=500 + e)
             for e, F, b in [(16, 9, 8), (16, 5, 2), (17, 4, 8), (14, 20, 8)]]
    scheds = [pk.Schedule(8, 8, 4, 0, 4), pk.Schedule(7, 0, 0, 2, 1), pk.Schedule(8, 8, 0, 0, 2),
              pk.Schedule(0, 0, 0, 0, 16)]
    packed = [torch.from_numpy(d["packed"]).to(dev) for d in insts]
    plan = pk.Plan([pk.Instance.from_synth(d) for d in insts], device=dev, schedules=scheds)
    plan.reset()
    plan.accumulate(packed)
    for i, (d, s, p) in enumerate(zip(insts, scheds, packed)):
        one = pk.Plan([pk.Instance.from_synth(d)], device=dev, schedules=[s])
        one.reset()
        one.accumulate(p)
        assert torch.equal(plan.spectra(i)[0], one.spectra()[0]), i


def test_tuner_cache(env, tmp_path, monkeypatch):
    torch, pk, dev = env
    from paper_1412_1256_amd import autotune
    path = str(tmp_path / "tune.json")
    monkeypatch.setenv(autotune.CACHE_ENV, path)
    inst = pk.Instance(fft_len=1 << 16, bits=8)
    say("autotune 2^16 int8")
    best, timings = autotune.tune(inst, device=dev, frames=16, reps=3)
    cands = pk.schedule_candidates(inst)
    assert best in cands and len(timings) == len(cands)
    d = json.load(open(path))
    key = autotune.cache_key(inst, dev)
    assert d[key]["schedule"] == {"log2_n1": best.log2_n1, "colpass_cols": best.colpass_cols,
                                  "rowpass_frames": best.rowpass_frames, "col_wg_per_cu": best.col_wg_per_cu,
                                  "rowpass_slots": best.rowpass_slots, "single_pass": best.single_pass}
    assert d[key]["ms"] == min(timings.values())

    def boom(*a, **k):
        raise AssertionError("timed again despite the cache")

    monkeypatch.setattr(autotune, "time_schedule", boom)
    assert autotune.best_schedule(inst, device=dev) == best
    plan = pk.Plan([inst], device=dev, tune=True)
    assert plan.schedules == [best]
