"""The batched-product autotuner: picks a candidate, caches it, and the tuned
configuration still matches the oracle."""
import json

import numpy as np
import pytest

from paper_2312_09763_amd import matvis as mv
from paper_2312_09763_amd import synth

from helpers import TOL, errors, gpu_simulate, grid_as_used, oracle_vis, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_autotune_picks_cached_candidate_and_stays_accurate(tmp_path, precision):
    wl = synth.workload(2, n_src=3001, n_time=5, n_freq=3)
    cfg = mv.config_for(wl, precision)
    d = mv.device_inputs(wl, precision)
    cache = str(tmp_path / "tune.json")
    tuned, ms = mv.autotune(cfg, **d, cache_path=cache)
    say(f"autotune {precision}: ksplit={tuned.ksplit} batch_time={tuned.batch_time} unfused={tuned.unfused} {ms:.3f} ms")
    # 0: the library's own choice, also a candidate
    allowed = {"fp32": {0, 1024, 2048}, "bf16x3": {0, 2048, 4096, 8192}}[precision]
    assert tuned.ksplit in allowed and tuned.batch_time in (0, 2, 4) and ms > 0
    text = open(cache).read()
    entries = json.loads(text)
    assert len(entries) == 1
    (key, val), = entries.items()
    assert key.startswith("gfx950|N256|ax2|src3001|t5|f3")
    assert val["ksplit"] == tuned.ksplit
    # a second call is answered from the cache
    tuned2, ms2 = mv.autotune(cfg, **d, cache_path=cache)
    assert (tuned2.ksplit, tuned2.batch_time, tuned2.unfused) == (tuned.ksplit, tuned.batch_time, tuned.unfused)
    assert abs(ms2 - ms) < 1e-3
    # the tuned configuration is still within the precision's tolerance
    V = gpu_simulate(wl, precision, ksplit=tuned.ksplit, batch_time=tuned.batch_time, unfused=tuned.unfused)
    ref = oracle_vis(wl, grid=grid_as_used(wl, precision))
    ef, ec = errors(V, ref)
    say(f"  err_F={ef:.3e} err_CS={ec:.3e}")
    assert ef <= TOL[precision] and ec <= TOL[precision]
