"""Tuning-cache lookups on the host (no GPU): the nearest tuned qubit count,
the tile width capped for the block size, and the fused configuration kept
beside a non-fused winner."""
from paper_1908_07187_amd import autotune

CACHE = {
    "gfx950|c128|n22": {"fusion": 0, "stages": 1, "ms_per_gate": 0.005,
                        "fused": {"fusion": 5, "mfma_cols": 64, "mfma_areg": 1, "mfma_waves": 8, "mfma_lds": 0,
                                  "ms_per_gate": 0.007}},
    "gfx950|c128|n30": {"fusion": 5, "mfma_cols": 64, "mfma_lds": 0, "ms_per_gate": 0.9},
    "gfx950|c64|n26": {"fusion": 0, "stages": 1, "ms_per_gate": 0.03},
}


def test_lookup_takes_the_nearest_qubit_count():
    assert autotune.lookup(24, "c128", CACHE, device="gfx950")["stages"] == 1
    assert autotune.lookup(29, "c128", CACHE, device="gfx950")["fusion"] == 5
    assert autotune.lookup(20, "c128", CACHE, device="gfx942") is None


def test_tile_width_capped_also_in_the_kept_fused_entry():
    # complex128 5-qubit blocks have register tiles of at most 32 columns
    assert autotune.lookup(30, "c128", CACHE, device="gfx950")["mfma_cols"] == 32
    kept = autotune.lookup(22, "c128", CACHE, device="gfx950")["fused"]
    assert kept["mfma_cols"] == 32 and kept["fusion"] == 5


def test_fused_config():
    assert autotune.fused_config(None) is None
    winner = autotune.lookup(30, "c128", CACHE, device="gfx950")
    assert autotune.fused_config(winner) is winner
    kept = autotune.fused_config(autotune.lookup(22, "c128", CACHE, device="gfx950"))
    assert kept["fusion"] == 5 and "stages" not in kept
    # a non-fused winner without a kept fused entry (an older cache) has none
    assert autotune.fused_config(autotune.lookup(26, "c64", CACHE, device="gfx950")) is None
