"""Seeded Gaussian random fields for the synthetic reservoir properties.

Recipe: squared-exponential covariance C(r) = exp(-sum_d (r_d / l_d)^2), produced
by FFT filtering of white noise on a grid padded by 3 correlation lengths per axis
(to suppress wrap-around), cropped, then empirically standardised to zero mean and
unit variance.  The spectral density of C in 1-D is proportional to
exp(-k^2 l^2 / 4), so the amplitude filter is exp(-k^2 l^2 / 8).

The paper's own heterogeneous field (SPE10 Model 2, Sec. 6.2) is not available;
these fields stand in for it.
"""
import numpy as np


def gaussian_field(rng, shape_zyx, h, lengths_zyx):
    """Standardised GRF on a grid of `shape_zyx` cells of size h (array order z, y, x).

    lengths_zyx: correlation lengths (m) per axis.  Returns float64 array of shape
    shape_zyx whose flattening (C order) is lexicographic with x fastest.
    """
    shape = tuple(int(n) for n in shape_zyx)
    pad = tuple(n + int(np.ceil(3.0 * l / h)) for n, l in zip(shape, lengths_zyx))
    noise = rng.standard_normal(pad)
    spec = np.fft.rfftn(noise)
    kz = 2.0 * np.pi * np.fft.fftfreq(pad[0], d=h)
    ky = 2.0 * np.pi * np.fft.fftfreq(pad[1], d=h)
    kx = 2.0 * np.pi * np.fft.rfftfreq(pad[2], d=h)
    lz, ly, lx = lengths_zyx
    filt = (np.exp(-(kz[:, None, None] * lz) ** 2 / 8.0)
            * np.exp(-(ky[None, :, None] * ly) ** 2 / 8.0)
            * np.exp(-(kx[None, None, :] * lx) ** 2 / 8.0))
    field = np.fft.irfftn(spec * filt, s=pad, axes=(0, 1, 2))[: shape[0], : shape[1], : shape[2]]
    field = field - field.mean()
    sd = field.std()
    if sd > 0:
        field = field / sd
    return np.ascontiguousarray(field)


def gaussian_field_2d(rng, shape_yx, h, lengths_yx):
    """2-D standardised GRF (one layer), same recipe as gaussian_field."""
    f = gaussian_field(rng, (1,) + tuple(shape_yx), h, (h,) + tuple(lengths_yx))
    return f[0]
