"""Seeded synthetic input generators shared by the tests, the benchmark and the oracle.

This module holds none of the lattice method's arithmetic: it only draws initial
velocity fields, material-parameter fields, probe locations and finite-difference
directions from fixed seeds, so that the HIP library and the FP64 oracle are fed the same
inputs.  Fields that the library consumes in single precision (mu, lambda, body force) are
returned already rounded to float32 and widened back to float64, so both sides see the
identical values.

The workloads mirror the paper's test problems (Sec. 4-5 use analytic fields on square
periodic or bounded domains); the random fields stand in for the smooth initial data
those problems use, at the grid sizes the benchmark needs.
"""
import numpy as np

__all__ = [
    "shear_wave_v0", "gaussian_random_field", "lognormal_field", "random_probes",
    "fd_directions", "round_f32", "uniform_body",
]


def round_f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def shear_wave_v0(nx, ny, amp=1e-3):
    """v1 = amp sin(2 pi (b + 1/2) / ny), v2 = 0 on a cell-centred grid: a transverse wave
    travelling along Y (a standing S-wave on a periodic square)."""
    b = np.arange(ny, dtype=np.float64)
    v = np.zeros((2, ny, nx))
    v[0] = (amp * np.sin(2.0 * np.pi * (b + 0.5) / ny))[:, None]
    return v


def _wavenumbers(nx, ny):
    kx = 2.0 * np.pi * np.fft.rfftfreq(nx)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny)
    return kx[None, :], ky[:, None]


def _filtered_noise(nx, ny, seed, amplitude_of_k, zero_nyquist):
    import scipy.fft as sfft
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((ny, nx))
    W = sfft.rfft2(w, workers=8)
    del w
    kx, ky = _wavenumbers(nx, ny)
    kk = np.sqrt(kx * kx + ky * ky)
    with np.errstate(divide="ignore"):
        amp = amplitude_of_k(kk)
    amp[0, 0] = 0.0
    if zero_nyquist:
        if nx % 2 == 0:
            amp[:, -1] = 0.0
        if ny % 2 == 0:
            amp[ny // 2, :] = 0.0
    W *= amp
    return sfft.irfft2(W, s=(ny, nx), workers=8)


def gaussian_random_field(nx, ny, seed, rms, spectral_slope=-3.0):
    """Real Gaussian random field with power spectrum ~ |k|^slope: white noise from
    numpy's PCG64 generator seeded with ``seed``, filtered by |k|^(slope/2) with the mean
    and Nyquist modes removed, rescaled to the requested rms."""
    g = _filtered_noise(nx, ny, seed, lambda k: k ** (0.5 * spectral_slope), True)
    g *= rms / np.sqrt(np.mean(g * g))
    return g


def lognormal_field(nx, ny, seed, median, sigma_log=0.3, corr_len=32.0):
    """median * exp(sigma_log g), g a smooth Gaussian field with covariance
    exp(-r^2 / (2 l^2)) (filter exp(-|k|^2 l^2 / 4)) normalised to mean 0 and std 1.
    Rounded to float32."""
    g = _filtered_noise(nx, ny, seed, lambda k: np.exp(-0.25 * (k * corr_len) ** 2), False)
    g -= g.mean()
    g /= g.std()
    return round_f32(median * np.exp(sigma_log * g))


def uniform_body(nx, ny, b):
    out = np.empty((2, ny, nx))
    out[0] = b[0]
    out[1] = b[1]
    return round_f32(out)


def random_probes(nx, ny, count, seed, margin=2):
    """``count`` distinct cells drawn uniformly, at least ``margin`` cells away from every
    side of the grid.  Returns (ys, xs) int arrays."""
    rng = np.random.default_rng(seed)
    cand = (ny - 2 * margin) * (nx - 2 * margin)
    idx = rng.choice(cand, size=count, replace=False)
    ys = margin + idx // (nx - 2 * margin)
    xs = margin + idx % (nx - 2 * margin)
    return ys.astype(np.int64), xs.astype(np.int64)


def fd_directions(shapes, count, seed):
    """``count`` random directions, standard normal per entry, for each array shape in
    ``shapes`` (a dict name -> shape)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        out.append({k: rng.standard_normal(s) for k, s in shapes.items()})
    return out
