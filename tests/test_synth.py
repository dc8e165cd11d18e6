"""The seeded generator follows the published SplitMix64 definition."""

import numpy as np

from paper_2011_10658_amd import synth


def test_splitmix64_reference_output():
    # first output of SplitMix64 started from state 0 (state += gamma, mix)
    assert int(synth._mix(np.uint64(0x9E3779B97F4A7C15))) == 0xE220A8397B1DCDAF


def test_counter_streams():
    a = synth.sym_uniform(3, 7, 100)
    b = synth.sym_uniform(3, 7, 50)
    assert np.array_equal(a[:50], b)
    assert np.all((a >= -1) & (a < 1))
    assert not np.array_equal(a, synth.sym_uniform(3, 8, 100))
    z = synth.normal(1, 2, 20001)
    assert abs(z.mean()) < 0.03 and abs(z.std() - 1) < 0.03


def test_random_composition():
    for s in range(20):
        sizes = synth.random_composition(s, 5, 64, 7)
        assert len(sizes) == 7 and sum(sizes) == 64 and min(sizes) >= 1
