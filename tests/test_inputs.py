"""The seeded input generator shared by the oracle and the GPU path.

SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) is pinned to its published
first outputs from state 0; the derived draws are checked for range and
distribution.  CPU only."""
import numpy as np

from paper_1511_04633_amd import inputs


def test_splitmix64_known_answers():
    """From state 0 the generator's first three outputs are the published
    0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f; the counter
    form gives draw k of any offset without the earlier ones."""
    v = inputs.splitmix64(0, 3)
    assert [int(x) for x in v] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert int(inputs.splitmix64(0, 1, offset=2)[0]) == 0x06C45D188009454F
    assert np.array_equal(inputs.splitmix64(7, 10)[4:], inputs.splitmix64(7, 6, offset=4))


def test_uniform_and_theta_noise():
    u = inputs.uniform01(20151115, 200_000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 3e-3 and abs(u.var() - 1 / 12) < 2e-3
    th = inputs.theta_noise(16, 20151115)
    assert th.shape == (16 ** 3,) and np.abs(th).max() <= 1e-6
    assert np.array_equal(th, inputs.theta_noise(16, 20151115))       # seeded
    assert not np.array_equal(th, inputs.theta_noise(16, 20151116))


def test_batch_cases_cover_the_configured_ranges():
    cases = inputs.batch_cases(1511, 64)
    assert len(cases) == 64
    assert {c["n"] for c in cases} == {32, 48, 64, 80, 96}
    assert {c["wall_type"] for c in cases} == {1, 2, 3}
    ra = np.array([c["ra"] for c in cases])
    assert ra.min() >= 1e3 and ra.max() <= 1e6
    assert cases == inputs.batch_cases(1511, 64)
