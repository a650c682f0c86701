"""Host logic of the FFT convolution pipeline (no GPU): the FFT-friendly
sizes and the result shape."""
from paper_1608_00099_amd import fftconv


def _is_smooth(m):
    for p in (2, 3, 5):
        while m % p == 0:
            m //= p
    return m == 1


def test_good_size_is_the_least_5_smooth_bound():
    for n in range(1, 2000):
        g = fftconv.good_size(n)
        assert g >= n and _is_smooth(g)
        assert all(not _is_smooth(m) for m in range(n, g))


def test_conv_shape():
    assert fftconv.conv_shape((256, 8), (256, 8)) == (511, 15)
    assert fftconv.conv_shape((), ()) == ()
