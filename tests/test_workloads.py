"""The shared input generator reproduces SplitMix64's published first output."""
import workloads


def test_splitmix64_reference_value():
    # first output of SplitMix64 seeded with 0 (Steele, Lea & Flood 2014)
    assert workloads.splitmix64(0) == 0xE220A8397B1DCDAF


def test_batch_draws_in_range():
    jobs = workloads.batch_jobs(64)
    assert len({j.seed for j in jobs}) == 64
    assert all(4.0 <= j.h < 20.0 and 0.001 <= j.g < 0.05 for j in jobs)
    assert jobs == workloads.batch_jobs(64)
