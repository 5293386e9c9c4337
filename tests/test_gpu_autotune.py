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
    say(f"autotune {precision}: tile={tuned.tile} ksplit={tuned.ksplit} src_chunk={tuned.src_chunk} "
        f"batch_time={tuned.batch_time} unfused={tuned.unfused} {ms:.3f} ms")
    # candidates: 0 (the library's choice) and, on the product over sources, 2, 4, 1/2
    # and 1/4 times the path's default k-split (8192 FP32, 20480 BF16X3), the
    # 64-antenna forming split, times per batch 1..8 (<= 5 here); no chunk below 3001 sources
    allowed = {"fp32": {0, 16384, 32768, 4096, 2048}, "bf16x3": {0, 40960, 81920, 10240, 5120}}[precision]
    assert tuned.ksplit in allowed and tuned.batch_time in (0, 1, 2, 4) and tuned.tile in (0, 2)
    assert tuned.src_chunk == 0 and ms > 0
    text = open(cache).read()
    entries = json.loads(text)
    assert len(entries) == 1
    (key, val), = entries.items()
    assert key == f"gfx950|path3|N256|ax2|nb1|fl0|src2^11|t5|f3|p{ {'fp32': 1, 'bf16x3': 2}[precision] }|b1"
    assert (val["ksplit"], val["tile"], val["src_chunk"]) == (tuned.ksplit, tuned.tile, tuned.src_chunk)
    # a second call is answered from the cache
    tuned2, ms2 = mv.autotune(cfg, **d, cache_path=cache)
    assert (tuned2.ksplit, tuned2.batch_time, tuned2.unfused, tuned2.tile, tuned2.src_chunk) == \
        (tuned.ksplit, tuned.batch_time, tuned.unfused, tuned.tile, tuned.src_chunk)
    assert abs(ms2 - ms) < 1e-3
    # the tuned configuration is still within the precision's tolerance
    V = gpu_simulate(wl, precision, ksplit=tuned.ksplit, batch_time=tuned.batch_time, unfused=tuned.unfused,
                     tile=tuned.tile, src_chunk=tuned.src_chunk)
    ref = oracle_vis(wl, grid=grid_as_used(wl, precision))
    ef, ec = errors(V, ref)
    say(f"  err_F={ef:.3e} err_CS={ec:.3e}")
    assert ef <= TOL[precision] and ec <= TOL[precision]


@pytest.mark.parametrize("tile", [2, 3])
def test_forming_split_variants_agree(tile):
    """The kernel variants the autotuner picks among give the same visibilities:
    the forming split only reschedules work, so the result is bitwise the same."""
    wl = synth.workload(2, n_ant=128, n_src=700, n_time=2, n_freq=2)
    V0 = gpu_simulate(wl, "bf16x3")
    V1 = gpu_simulate(wl, "bf16x3", tile=tile)
    say(f"forming split {32 * tile} antennas: bitwise equal {np.array_equal(V0, V1)}")
    assert np.array_equal(V0, V1)
    ws = synth.workload(3, n_src=3072, n_time=1, n_freq=2)
    for t in (2, 4):
        assert np.array_equal(gpu_simulate(ws, "bf16x3"), gpu_simulate(ws, "bf16x3", tile=t))


def test_autotune_learned_beam(tmp_path):
    import torch
    wl = synth.workload(2, n_ant=96, n_src=2000, n_time=2, n_freq=2)
    cfg = mv.config_for(wl, "bf16x3", beam_mode="surrogate")
    d = mv.device_inputs(wl, "bf16x3")
    P = torch.from_numpy(synth.surrogate_init(0)).cuda()
    tuned, ms = mv.autotune(cfg, **d, cache_path=str(tmp_path / "t.json"), surrogate=P)
    say(f"autotune with the learned beam: tile={tuned.tile} ksplit={tuned.ksplit} {ms:.3f} ms")
    assert ms > 0 and tuned.beam_mode == "surrogate"


@pytest.mark.parametrize("variant", [16])
@pytest.mark.parametrize("n_ant", [301, 350])
def test_block_pair_kernel_variants_match_oracle(variant, n_ant):
    """The block-pair kernel variant of the product over sources (tile bit 4: the
    two-sided square-root weights) against the oracle, on three 128-antenna blocks
    with a short last block (45 or 94 antennas), beside the default kernel."""
    wl = synth.workload(2, n_ant=n_ant, n_src=600, n_time=1, n_freq=2)
    V = gpu_simulate(wl, "bf16x3", tile=variant)
    V0 = gpu_simulate(wl, "bf16x3")
    ref = oracle_vis(wl, grid=grid_as_used(wl, "bf16x3"))
    ef, ec = errors(V, ref)
    ef0, ec0 = errors(V0, ref)
    say(f"block-pair variant {variant}, {n_ant} antennas: err_F={ef:.3e} err_CS={ec:.3e} "
        f"(default kernel {ef0:.3e} / {ec0:.3e})")
    assert ef <= 1e-5 and ec <= 1e-5


@pytest.mark.parametrize("split", [0, 2, 4])
def test_stage_depth_variant_is_bitwise_the_same(split):
    """16 sources per stage on the BF16X3 three-block path (tile bit 6) against the
    default 32: the MFMAs of either stage depth accumulate in the same source order,
    so V is bitwise the same; with each forming split, and against the oracle."""
    ws = synth.workload(3, n_src=3072, n_time=2, n_freq=2)
    V0 = gpu_simulate(ws, "bf16x3", tile=split | 64)
    V1 = gpu_simulate(ws, "bf16x3", tile=split)
    say(f"stage depth 16 against 32, forming split {split}: bitwise equal {np.array_equal(V0, V1)}")
    assert np.array_equal(V0, V1)
    ef, ec = errors(V1, oracle_vis(ws, grid=grid_as_used(ws, "bf16x3")))
    say(f"  err_F={ef:.3e} err_CS={ec:.3e}")
    assert ef <= TOL["bf16x3"] and ec <= TOL["bf16x3"]
