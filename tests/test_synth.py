"""Pins of the seeded input generators (no GPU): the counter-based
generator behind a setup started without test vectors."""
import numpy as np

import synth


def _one(ctr, key):
    r = synth.philox4x32_10([[c] for c in ctr], [[k] for k in key])
    return [int(x[0]) for x in r]


def test_philox4x32_10_known_answers():
    """The known-answer vectors published with the Philox4x32-10 reference
    implementation (Random123): zero counter and key, all-ones counter and
    key, and the hexadecimal digits of pi."""
    assert _one([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert _one([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]
    assert _one([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0]) == \
        [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


def test_philox_gaussians_layout_and_moments():
    L = (4, 4, 4, 4)
    g = synth.philox_gaussian_spinors(L, 8, 5)
    assert g.shape == (8, 4, 4, 4, 4, 4, 3)
    # element i of the flat array is the Box-Muller pair of counter i
    i = 1234
    x = synth.philox4x32_10([[i], [0], [0], [0]], [[5], [0]])
    u1 = (int(x[0][0]) >> 5) * 2.0 ** -27 + (int(x[1][0]) >> 6) * 2.0 ** -53
    u2 = (int(x[2][0]) >> 5) * 2.0 ** -27 + (int(x[3][0]) >> 6) * 2.0 ** -53
    rho = np.sqrt(-2.0 * np.log(1.0 - u1))
    assert g.reshape(-1)[i] == rho * np.cos(2 * np.pi * u2) + 1j * rho * np.sin(2 * np.pi * u2)
    # unit-variance independent real and imaginary parts, like gaussian_spinors
    n = g.size
    assert abs(g.real.mean()) < 5 / np.sqrt(n) and abs(g.imag.mean()) < 5 / np.sqrt(n)
    assert abs(g.real.var() - 1) < 0.05 and abs(g.imag.var() - 1) < 0.05
    assert abs(np.mean(g.real * g.imag)) < 5 / np.sqrt(n)
    # the seed's high word enters the key
    assert not np.array_equal(synth.philox_gaussian_spinors(L, 1, 5), synth.philox_gaussian_spinors(L, 1, 5 + (1 << 32)))


def test_uneven_instances_recipe():
    """The batched-serving recipe: shapes from the four uneven lattices,
    parameters in their stated ranges, 2^4 blocks exactly for 12^4 (an even
    number of blocks per direction), deterministic in the seed."""
    a = synth.uneven_instances(64, 3)
    b = synth.uneven_instances(64, 3)
    assert a == b
    assert synth.uneven_instances(64, 4) != a
    assert {i["L"] for i in a} == set(synth.UNEVEN_SHAPES)
    for i in a:
        assert 0.3 <= i["eps"] <= 0.5 and -0.2 <= i["m0"] <= -0.05 and i["ntv"] == 16
        assert i["block"] == ((2, 2, 2, 2) if i["L"][0] == 12 else (4, 4, 4, 4))
        for L, bs in zip(i["L"], i["block"]):
            assert L % bs == 0 and (L // bs) % 2 == 0
    seeds = [s for i in a for s in (i["gauge_seed"], i["setup_seed"], i["rhs_seed"])]
    assert len(set(seeds)) == len(seeds)
