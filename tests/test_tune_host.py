"""Host checks of the library's tuning table (no GPU): keys, set/get, the JSON
cache file round trip, loading by BTA_TUNE_CACHE in a fresh process, and the
environment override of the factor's lookahead (the schedule the factor plan
would run, replayed on the host)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def tune():
    from paper_2503_17528_amd import autotune, bta

    if not os.path.exists(bta.LIB_PATH):
        pytest.fail("libbta.so is not built (run __graft_entry__.build())")
    autotune.clear()
    yield autotune
    autotune.clear()


def test_key_names_arch_op_shape_knob(tune):
    k = tune.key("factor", 2048, 8, "look")
    assert k.endswith("|factor|b=2048|a=8|look")
    assert k.split("|")[0].startswith("gfx")


def test_set_get_dump(tune):
    k = tune.key("factor", 512, 4, "look")
    assert tune.get_entry(k) is None
    tune.set_entry(k, 6)
    assert tune.get_entry(k) == 6
    assert tune.table()[k] == 6
    with pytest.raises(ValueError):
        tune.set_entry('bad"key', 1)


def test_json_round_trip(tune, tmp_path):
    k1, k2 = tune.key("factor", 1024, 256, "look"), tune.key("factor", 1024, 256, "cached")
    tune.set_entry(k1, 12)
    tune.set_entry(k2, 1)
    path = str(tmp_path / "tune.json")
    tune.save(path)
    data = json.load(open(path))
    assert data["entries"][k1] == 12 and data["entries"][k2] == 1
    tune.clear()
    assert tune.get_entry(k1) is None
    tune.load(path)
    assert tune.get_entry(k1) == 12 and tune.get_entry(k2) == 1
    with pytest.raises(OSError):
        tune.load(str(tmp_path / "missing.json"))


def _fresh(code, env):
    e = dict(os.environ)
    e.update(env)
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=e, capture_output=True, text=True, timeout=120)


def test_cache_file_loaded_on_first_use(tmp_path):
    path = str(tmp_path / "t.json")
    code = ("from paper_2503_17528_amd import autotune as t; k=t.key('factor',256,4,'look'); "
            "print(t.get_entry(k))")
    with open(path, "w") as f:
        f.write('{"entries": {"gfx950|factor|b=256|a=4|look": 3}}')
    r = _fresh(code, {"BTA_TUNE_CACHE": path})
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == "3"


def test_lookahead_sources_reach_the_factor_plan():
    """Precedence of the factor's tunables as the plan sees them: the tuning
    table beats the default, the environment beats the table, the internal
    override beats the environment; b=2048 keeps every value below T-1."""
    code = ("import ctypes; from paper_2503_17528_amd import bta, autotune as t; L=bta.lib(); "
            "lk=ctypes.c_int(0); ca=ctypes.c_int(0); "
            "q=lambda: (L.bta_internal_factor_plan_knobs(ctypes.c_int64(8),ctypes.c_int64(2048),ctypes.c_int64(8),"
            "ctypes.byref(lk),ctypes.byref(ca)), (lk.value, ca.value))[1]; "
            "r=[q()]; t.set_entry(t.key('factor',2048,8,'look'),5); t.set_entry(t.key('factor',2048,8,'cached'),1); "
            "r.append(q()); L.bta_internal_factor_lookahead(3); r.append(q()); "
            "L.bta_internal_factor_lookahead(0); r.append(q()); print(r)")
    r = _fresh(code, {})
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == "[(8, 0), (5, 1), (3, 1), (5, 1)]"
    r = _fresh(code, {"BTA_FACTOR_LOOKAHEAD": "12", "BTA_FACTOR_CACHED": "0"})
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == "[(12, 0), (12, 0), (3, 0), (12, 0)]"
