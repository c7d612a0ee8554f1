"""Seeded random fields (NumPy PCG64) standing in for the paper's permeability maps.

The paper's Case-1..4 fields (an H-shaped zone shown only in a figure, an
MRST geostatistical field, SPE10) are not available, so the workloads use
fields with the same scales and heterogeneity built here.

Gaussian random field: white noise is filtered in Fourier space on a grid
padded to twice the size (so the periodic FFT does not wrap correlation
across opposite faces) with the kernel exp(-2 r^2 / l^2), whose
autocorrelation is exp(-r^2 / l^2); the crop is shifted to zero mean and
scaled to unit variance.
"""
import numpy as np


def gaussian_field(shape, corr_len, seed):
    """Zero-mean, unit-variance correlated field of the given shape (x fastest last axis)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = tuple(int(s) for s in shape)
    pad = tuple(2 * s for s in shape)
    noise = rng.standard_normal(pad)
    # squared distance in cells on the periodic padded grid
    r2 = np.zeros(pad)
    for ax, n in enumerate(pad):
        d = np.minimum(np.arange(n), n - np.arange(n)).astype(np.float64)
        sh = [1] * len(pad)
        sh[ax] = n
        r2 = r2 + (d ** 2).reshape(sh)
    kern = np.exp(-2.0 * r2 / (corr_len ** 2))
    f = np.fft.ifftn(np.fft.fftn(noise) * np.fft.fftn(kern)).real
    f = f[tuple(slice(0, s) for s in shape)]
    f = f - f.mean()
    sd = f.std()
    return f / sd if sd > 0 else f


def lognormal_perm(shape, mean_perm, sigma, corr_len, seed):
    """K = exp(ln(mean_perm) + sigma * G), same units as mean_perm."""
    return np.exp(np.log(mean_perm) + sigma * gaussian_field(shape, corr_len, seed))


def layered_perm(nx, ny, nz, kmin, kmax, sigma, corr_len, seed):
    """Per-layer mean drawn log-uniformly in [kmin, kmax]; each layer is an
    independent 2D log-normal field around its mean.  Returns (nz, ny, nx)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    means = np.exp(rng.uniform(np.log(kmin), np.log(kmax), size=nz))
    out = np.empty((nz, ny, nx))
    for k in range(nz):
        g = gaussian_field((ny, nx), corr_len, seed * 1000 + k + 1)
        out[k] = np.exp(np.log(means[k]) + sigma * g)
    return out


def channel_perm(nx, ny, nz, k_bg, k_ch, nchan, seed):
    """Background k_bg with nchan sinusoidal channels of k_ch running along x.

    Each channel: centre line y0 + A sin(2 pi x / wavelength + phase), half
    width w/2 in y, occupying a vertical band of layers.  Returns (nz, ny, nx).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.full((nz, ny, nx), float(k_bg))
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    for _ in range(nchan):
        y0 = rng.uniform(0, ny)
        amp = rng.uniform(4, 12)
        wl = rng.uniform(24, 96)
        ph = rng.uniform(0, 2 * np.pi)
        width = int(rng.integers(3, 7))
        band = int(rng.integers(4, 9))
        z0 = int(rng.integers(0, max(1, nz - band + 1)))
        yc = y0 + amp * np.sin(2 * np.pi * x / wl + ph)           # (nx,)
        mask2 = np.abs(y[:, None] - yc[None, :]) <= 0.5 * width  # (ny, nx)
        out[z0:z0 + band][:, mask2] = k_ch
    return out


def hzone_mask(nx, ny):
    """Cells of an H-shaped zone on the unit square (x fastest): two bars at
    x in [0.20, 0.35] and [0.65, 0.80] for y in [0.15, 0.85], joined by a
    crossbar x in [0.35, 0.65], y in [0.425, 0.575] (cell centres)."""
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)
    bars = (((X >= 0.20) & (X <= 0.35)) | ((X >= 0.65) & (X <= 0.80))) & (Y >= 0.15) & (Y <= 0.85)
    cross = (X > 0.35) & (X < 0.65) & (Y >= 0.425) & (Y <= 0.575)
    return bars | cross
