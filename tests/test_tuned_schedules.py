"""The committed schedule cache holds an entry for every configuration
bench.py measures, so the bench and the GPU parity tests of those
configurations read the same schedules instead of tuning again."""
from tuned_keys import TUNED, bench_batch_key, bench_system_keys, read_tuned


def test_cache_has_every_bench_configuration():
    tuned = read_tuned()
    for what, key in bench_system_keys().items():
        assert key in tuned, f"{what}: {key} missing from {TUNED}"
        L, cc, nt, G, T, nbuf = tuned[key]
        assert L & (L - 1) == 0 and cc in (2, 4, 8) and nt % 64 == 0 and G >= 1
        assert 1 <= T <= 32 and nbuf in (1, 2)
    key = bench_batch_key()
    assert key in tuned and len(tuned[key]) == 4, f"batch: {key[:60]}... missing from {TUNED}"
