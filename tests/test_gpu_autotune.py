"""The autotuners on the GPU: the factor tuner times every candidate (median
of three runs) and records the fastest lookahead, load path and SUB delay, which the
next factorization then uses (checked against the oracle); the selected
inversion's split tuner likewise (the next selected inversion checked against
the oracle); the batched
selected inversion records its per-stage tile choices on first use; both
appear in the table dump and survive a save / load round trip."""
import numpy as np
import pytest

import oracle
from paper_2503_17528_amd import synth
from tests.gpu_util import TOL, errs, say, to_np

pytestmark = pytest.mark.gpu


def test_factor_tuner_and_batched_tuner(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_17528_amd import autotune, bta

    bta.lib()
    try:
        _run(torch, autotune, bta, tmp_path)
    finally:
        autotune.clear()  # later tests run with the built-in defaults


def _run(torch, autotune, bta, tmp_path):
    n, b, a = 6, 256, 4
    say(f"case autotune factor n={n} b={b} a={a}")
    times = autotune.tune_factor(n, b, a, looks=(1, 2, 3), cached=(0, 1), reps=3, log=say, sub_delays=(0, 1, 4))
    lc = {k: v for k, v in times.items() if k.startswith("look=")}
    sd = {k: v for k, v in times.items() if k.startswith("sub_delay=")}
    assert len(lc) == 6 and all(t > 0 for t in times.values())
    assert set(sd) == {"sub_delay=0", "sub_delay=1", "sub_delay=4"}
    look = autotune.get_entry(autotune.key("factor", b, a, "look"))
    cached = autotune.get_entry(autotune.key("factor", b, a, "cached"))
    delay = autotune.get_entry(autotune.key("factor", b, a, "sub_delay"))
    best = min(lc, key=lc.get)
    assert best == f"look={look},cached={cached}", (best, look, cached)
    assert min(sd, key=sd.get) == f"sub_delay={delay}", (sd, delay)

    # the tuned settings are the ones the next factorization runs with
    Q = synth.make_np(synth.workload(n, b, a), 3)
    F = oracle.pobtaf(Q["D"], Q["B"], Q["R"], Q["T"])
    D, B, R, T = (torch.from_numpy(Q[k]).to("cuda") for k in "DBRT")
    L = bta.factor(D, B, R, T)
    torch.cuda.synchronize()
    e = errs(dict(zip("DBRT", to_np(L[:4]))), {"D": F["LD"], "B": F["LB"], "R": F["LR"], "T": F["LT"]})
    say(f"   tuned factor vs oracle: {e}")
    assert max(e.values()) < TOL

    # the selected inversion's split count at a small b (64 output tiles: the split applies)
    n2, b2, a2 = 4, 512, 4
    say(f"case autotune selinv split n={n2} b={b2} a={a2}")
    st = autotune.tune_selinv_split(n2, b2, a2, reps=3, log=say)
    assert set(st) == {"split=1", "split=2", "split=3", "split=4"}
    sp = autotune.get_entry(autotune.key("selinv", b2, a2, "split"))
    assert f"split={sp}" == min(st, key=st.get)
    Q2 = synth.make_np(synth.workload(n2, b2, a2), 4)
    F2 = oracle.pobtaf(Q2["D"], Q2["B"], Q2["R"], Q2["T"])
    X2o = oracle.pobtasi(F2["LD"], F2["LB"], F2["LR"], F2["LT"])
    L2 = [torch.from_numpy(np.ascontiguousarray(F2[k])).to("cuda") for k in ("LD", "LB", "LR", "LT")]
    X2 = bta.selinv(*L2)
    torch.cuda.synchronize()
    e2 = errs(dict(zip("DBRT", to_np(X2))), {"D": X2o["XD"], "B": X2o["XB"], "R": X2o["XR"], "T": X2o["XT"]}, lower=())
    say(f"   tuned selinv (split {sp}) vs oracle: {e2}")
    assert max(e2.values()) < TOL

    # batched selected inversion: first use measures and records its stage choices
    mats = [synth.make_torch(synth.workload(4, 128, 2), 70 + k, "cuda") for k in range(3)]
    batch = bta.Batch(mats)
    batch.factor()
    batch.selinv()
    torch.cuda.synchronize()
    tab = autotune.table()
    stage_keys = [k for k in tab if "|selinv_batched[" in k and k.endswith("|tile128")]
    say(f"   table: {len(tab)} entries, {len(stage_keys)} batched stage classes")
    assert any(k.endswith(f"|factor|b={b}|a={a}|look") for k in tab)
    assert any(k.endswith(f"|selinv|b={b2}|a={a2}|split") for k in tab)
    assert stage_keys and all(tab[k] in (0, 1) for k in stage_keys)
    path = str(tmp_path / "tune.json")
    autotune.save(path)
    autotune.clear()
    autotune.load(path)
    assert autotune.table() == tab
