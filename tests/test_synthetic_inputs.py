"""The seeded input generators: the chunked float32 generator and the patch generator give exactly
the values of phi0 (site i takes draw i of the SplitMix64 stream), and the stream itself matches
the published SplitMix64 outputs for seed 0."""
import numpy as np

import synthetic as S


def test_splitmix64_reference_outputs():
    # first outputs of SplitMix64 started at state 0 (the generator's published test values)
    z = S.splitmix64(0, np.arange(3, dtype=np.uint64))
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_chunked_generator_equals_phi0():
    for shape, chunk in (((60, 70, 90), 1000), ((33, 65), 7), ((5, 1 << 12), 1 << 10)):
        a = S.phi0(shape, seed=5, amplitude=0.2)
        b = S.phi0_f32(shape, seed=5, amplitude=0.2, chunk=chunk, threads=4)
        assert b.dtype == np.float32 and np.array_equal(a, b.astype(np.float64))


def test_patch_generator_equals_phi0_with_wrap():
    a = S.phi0((60, 70, 90), seed=11)
    p = S.phi0_patch((60, 70, 90), (55, 65, 80), (9, 10, 20), seed=11)
    ref = a[np.ix_(np.arange(55, 64) % 60, np.arange(65, 75) % 70, np.arange(80, 100) % 90)]
    assert np.array_equal(p, ref)
    b = S.phi0((40, 24), seed=2)
    q = S.phi0_patch((40, 24), (-3, 20), (8, 8), seed=2)
    assert np.array_equal(q, b[np.ix_(np.arange(-3, 5) % 40, np.arange(20, 28) % 24)])
