"""Host logic of the autotuner: buckets, candidates and cache lookup."""
from paper_1912_08810_amd import autotune


def test_buckets_cover_the_instance_ranges():
    assert autotune.bucket_of(200, 10) == (0, 0)
    assert autotune.bucket_of(600, 20) == (0, 0)
    assert autotune.bucket_of(601, 21) == (1, 1)
    assert autotune.bucket_of(1500, 40) == (2, 2)
    assert autotune.bucket_of(5000, 90) == (2, 2)   # beyond the last edge: last bucket


def test_candidates_pair_tiles_with_chunks():
    c = autotune.candidates(0, 10)
    assert (10, 0) in c and (5, 8) in c
    assert len(c) == len(set(c)) == 9
    assert all(te >= 1 and ct in (0, 8, 16) for te, ct in c)


def test_params_for_reads_the_bucket_and_defaults_when_untuned():
    cache = {"gfx950/prec=2/Norb=10": {"1,2": {"tile_e": 7, "chunk_taps": 16}}}
    assert autotune.params_for(2, 10, 800, 35, cache) == (7, 16)
    assert autotune.tile_for(2, 10, 800, 35, cache) == 7
    assert autotune.params_for(2, 10, 300, 35, cache) == (0, 0)     # other bucket
    assert autotune.params_for(0, 10, 800, 35, cache) == (0, 0)     # other precision
    old = {"gfx950/prec=0/Norb=10": {"0,0": {"tile_e": 10}}}         # entry without chunk
    assert autotune.params_for(0, 10, 400, 15, old) == (10, 0)
