"""Brain-MRI-like phantoms and band-limited random velocity fields.

The paper evaluates on NIREP brain volumes resampled to 180x210x180 (Section 4);
that database is not available here, so seeded synthetic volumes of the same
kind stand in for it: intensities in [0, 1], up to three tissue classes
(0.2 / 0.5 / 0.8), an ellipsoidal head shell and random anisotropic blob
"structures", smoothed by a Gaussian of one voxel.

Layout: scalar fields are float64 arrays of shape (N0, N1, N2) in C order
(x2 fastest); vector fields are (3, N0, N1, N2).  The domain is the periodic
box [0, 2*pi)^3, so the grid spacing is h_d = 2*pi / N_d.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

TISSUE_CLASSES = (0.2, 0.5, 0.8)


@dataclass(frozen=True)
class WorkloadSpec:
    """One synthetic registration workload (grid, phantom recipe and solver constants)."""

    name: str
    n: tuple
    n_blobs: int
    sigma_range: tuple  # blob standard deviations, in voxels
    classes: bool  # blob amplitudes drawn from TISSUE_CLASSES (else U[0.3, 1])
    shells: int  # 1 = single shell at 0.5, 3 = nested tissue shells
    disp_vox: float  # target max |v0| in voxels (stands in for max displacement)
    alpha: float
    s: int
    nt: int
    sigma2: float = 1.0
    noise_sd: float = 0.01
    gn_iters: int = 10
    cg_iters: int = 20
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    "pair32": WorkloadSpec("pair32", (32, 32, 32), 6, (2.0, 5.0), False, 1, 2.0, 0.01, 2, 10),
    "pair128": WorkloadSpec("pair128", (128, 128, 128), 24, (4.0, 12.0), True, 1, 6.0, 0.0025, 2, 10),
    "head180x216x180": WorkloadSpec(
        "head180x216x180", (180, 216, 180), 40, (5.0, 15.0), True, 3, 8.0, 0.0025, 2, 16
    ),
    "pair256": WorkloadSpec("pair256", (256, 256, 256), 48, (8.0, 24.0), True, 1, 12.0, 0.0025, 2, 32),
}


def _periodic_offsets(n):
    """Per-axis signed voxel offsets from the box centre, wrapped to [-N/2, N/2)."""
    return [np.arange(N, dtype=np.float64) - N / 2.0 for N in n]


def _gaussian_smooth(f, sigma_vox):
    """Periodic Gaussian smoothing (standard deviation in voxels) by a Fourier multiplier."""
    n = f.shape
    k = [np.fft.fftfreq(N) * 2.0 * np.pi for N in n[:2]] + [np.fft.rfftfreq(n[2]) * 2.0 * np.pi]
    k2 = k[0][:, None, None] ** 2 + k[1][None, :, None] ** 2 + k[2][None, None, :] ** 2
    return np.fft.irfftn(np.fft.rfftn(f) * np.exp(-0.5 * sigma_vox**2 * k2), s=n, axes=(0, 1, 2))


def phantom(n, n_blobs, sigma_range, classes, seed, shells=1, smooth_vox=1.0):
    """Template image: ellipsoidal head shell(s) plus random anisotropic Gaussian blobs.

    The ellipsoid is centred in the box with semi-axes (0.38, 0.42, 0.36) * N.
    ``shells=1`` puts a shell 0.9 <= rho <= 1 at intensity 0.5; ``shells=3`` fills
    nested shells rho in [0.9, 1] -> 0.2, [0.75, 0.9) -> 0.5, [0, 0.75) -> 0.8.
    Blob centres are uniform inside rho < 0.8, per-axis sigmas U[sigma_range] voxels,
    amplitudes U[0.3, 1] or a tissue class.  Sum, clip to [0, 1], smooth.
    """
    n = tuple(int(x) for x in n)
    rng = np.random.default_rng(seed)
    off = _periodic_offsets(n)
    semi = np.array([0.38, 0.42, 0.36]) * np.array(n, dtype=np.float64)
    rho = np.sqrt(
        (off[0][:, None, None] / semi[0]) ** 2
        + (off[1][None, :, None] / semi[1]) ** 2
        + (off[2][None, None, :] / semi[2]) ** 2
    )
    img = np.zeros(n)
    if shells == 1:
        img[(rho >= 0.9) & (rho <= 1.0)] = 0.5
    elif shells == 3:
        img[(rho >= 0.9) & (rho <= 1.0)] = 0.2
        img[(rho >= 0.75) & (rho < 0.9)] = 0.5
        img[rho < 0.75] = 0.8
    else:
        raise ValueError("shells must be 1 or 3")
    for _ in range(n_blobs):
        # centre uniform in the ellipsoid rho < 0.8 (rejection sampling)
        while True:
            c = rng.uniform(-0.8, 0.8, size=3)
            if np.sum(c * c) < 0.64:
                break
        centre = c * semi + np.array(n) / 2.0
        sig = rng.uniform(sigma_range[0], sigma_range[1], size=3)
        amp = TISSUE_CLASSES[rng.integers(0, 3)] if classes else rng.uniform(0.3, 1.0)
        g = np.ones(n)
        for d in range(3):
            x = np.arange(n[d], dtype=np.float64)
            dx = (x - centre[d] + n[d] / 2.0) % n[d] - n[d] / 2.0  # periodic minimum image
            shape = [1, 1, 1]
            shape[d] = n[d]
            g = g * np.exp(-0.5 * (dx / sig[d]) ** 2).reshape(shape)
        img = img + amp * g
    img = np.clip(img, 0.0, 1.0)
    if smooth_vox > 0:
        img = _gaussian_smooth(img, smooth_vox)
    return img


def random_field(n, seed, kc=None, components=3):
    """I.i.d. N(0,1) per component and voxel, low-pass filtered by exp(-|k|^2 / (2 kc^2)).

    Wavenumbers are the integer ones of the [0, 2*pi)^3 box; ``kc`` defaults to N/16
    (smallest axis).  Returns float64 of shape (components, N0, N1, N2).
    """
    n = tuple(int(x) for x in n)
    rng = np.random.default_rng(seed)
    if kc is None:
        kc = max(1.0, min(n) / 16.0)
    k = [np.fft.fftfreq(N, 1.0 / N) for N in n[:2]] + [np.fft.rfftfreq(n[2], 1.0 / n[2])]
    k2 = k[0][:, None, None] ** 2 + k[1][None, :, None] ** 2 + k[2][None, None, :] ** 2
    filt = np.exp(-k2 / (2.0 * kc * kc))
    out = np.empty((components,) + n)
    for c in range(components):
        w = rng.standard_normal(n)
        out[c] = np.fft.irfftn(np.fft.rfftn(w) * filt, s=n, axes=(0, 1, 2))
    return out


def random_velocity(n, seed, disp_vox, kc=None):
    """Band-limited random v0 scaled so that max_x |v0(x)| equals ``disp_vox`` voxels.

    For a geodesic of unit time the displacement is of the order of v0, so this
    amplitude stands in for the requested maximum displacement.
    """
    v = random_field(n, seed, kc)
    h = 2.0 * np.pi / min(n)
    vmax = np.sqrt(np.max(np.sum(v * v, axis=0)))
    return v * (disp_vox * h / vmax)


def noise(n, seed, sd):
    """Additive Gaussian image noise with standard deviation ``sd`` (no clipping)."""
    rng = np.random.default_rng(seed)
    return sd * rng.standard_normal(tuple(int(x) for x in n))


def pair_seeds(i):
    """Seeds of pair i: template 1000+i, velocity 2000+i, noise 3000+i."""
    return 1000 + i, 2000 + i, 3000 + i
