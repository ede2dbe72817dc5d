"""Seeded synthetic inputs for the rigid-alignment workloads.

This module is shared by the FP64 oracle and by the GPU path's tests and
benchmark.  It holds only input generation: pixel images of Gaussian blobs,
random rigid poses, white noise and the shift lattice.  None of the
alignment method's arithmetic (Fourier transforms, quadrature, Bessel
functions, SVD, inner products) lives here.

Conventions (Section 2 of the paper, "Problem setup"):
  * an n x n image samples a function on [-1, 1]^2 with spacing dx = 2/n;
    pixel (i, j) sits at x = i*dx - 1, y = j*dx - 1, so the first array
    index runs along x and the origin is pixel (n/2, n/2);
  * positions, blob widths and shifts are given here in pixel units;
  * the rotation R_g turns image content counter-clockwise by g about the
    origin, the translation T_s moves image content by +s.

An image is made from a template B as A = T_s R_theta B plus noise.  Its
best alignment X(delta, gamma) = <R_gamma T_delta A, B> is then reached at
delta = -s and gamma = -theta (mod 2 pi).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class BlobSet:
    """Isotropic Gaussian blobs, pixel units, centred on pixel (n/2, n/2)."""

    centers: np.ndarray  # (nblob, 2)  (x, y) in px
    sigmas: np.ndarray  # (nblob,)     px
    amps: np.ndarray  # (nblob,)

    def moved(self, theta: float, shift) -> "BlobSet":
        """Blobs of T_shift R_theta applied to this set (rotate, then shift)."""
        c, s = math.cos(theta), math.sin(theta)
        rot = np.array([[c, -s], [s, c]])
        return BlobSet(self.centers @ rot.T + np.asarray(shift, dtype=np.float64),
                       self.sigmas.copy(), self.amps.copy())


def random_blobs(rng: np.random.Generator, nblob: int, disk_px: float = 8.0,
                 sigma_px=(1.0, 3.0)) -> BlobSet:
    """nblob blobs: sigma ~ U[sigma_px], centres area-uniform in a disk."""
    r = disk_px * np.sqrt(rng.random(nblob))
    phi = 2.0 * np.pi * rng.random(nblob)
    centers = np.stack([r * np.cos(phi), r * np.sin(phi)], axis=1)
    sigmas = rng.uniform(sigma_px[0], sigma_px[1], nblob)
    return BlobSet(centers, sigmas, np.ones(nblob))


def render(blobs: BlobSet, n: int) -> np.ndarray:
    """Sample the blob sum at the n x n pixel centres (FP64, [i][j], i = x)."""
    p = np.arange(n, dtype=np.float64) - n / 2
    img = np.zeros((n, n))
    for (cx, cy), s, a in zip(blobs.centers, blobs.sigmas, blobs.amps):
        gx = np.exp(-((p - cx) ** 2) / (2 * s * s))
        gy = np.exp(-((p - cy) ** 2) / (2 * s * s))
        img += a * np.outer(gx, gy)
    return img


def unit_l2_scale(img: np.ndarray) -> float:
    """Factor that gives the pixel image unit L2 norm on [-1,1]^2."""
    n = img.shape[0]
    dx = 2.0 / n
    return 1.0 / math.sqrt(dx * dx * float(np.sum(img * img)))


def shift_lattice(radius_px: float, spacing_px: float = 0.5) -> np.ndarray:
    """All points of a square lattice within a disk, ordered by (dx, dy).

    Points with dx^2 + dy^2 <= radius^2 are kept (boundary included); the
    test is done in lattice units with integers so no point is lost to
    rounding.  Returns (N, 2) float64 pixel shifts.
    """
    rl = radius_px / spacing_px
    ri = int(math.floor(rl + 1e-9))
    r2 = rl * rl
    pts = []
    for i in range(-ri, ri + 1):
        for j in range(-ri, ri + 1):
            if i * i + j * j <= r2 + 1e-9:
                pts.append((i * spacing_px, j * spacing_px))
    return np.array(pts, dtype=np.float64)


def area_uniform_disk(rng: np.random.Generator, radius: float):
    r = radius * math.sqrt(rng.random())
    phi = 2.0 * math.pi * rng.random()
    return np.array([r * math.cos(phi), r * math.sin(phi)])


@dataclasses.dataclass
class AlignmentSet:
    """Templates, images and the ground truth that made the images."""

    n: int
    templates: np.ndarray  # (nB, n, n) float64
    images: np.ndarray  # (nA, n, n) float64
    template_blobs: list
    image_blobs: list  # noise-free moved blobs (scaled like the template)
    scales: np.ndarray  # (nB,) unit-L2 factor applied to each template
    true_template: np.ndarray  # (nA,) int
    true_theta: np.ndarray  # (nA,) rotation applied to the template
    true_shift: np.ndarray  # (nA, 2) shift applied after the rotation (px)
    noise_sigma: np.ndarray  # (nA,)
    clean: np.ndarray | None = None  # (nA, n, n) noise-free images if kept


def make_alignment_set(seed: int, n: int, n_templates: int, n_images: int,
                       nblob: int, shift_radius_px: float, snr: float | None,
                       disk_px: float = 8.0, sigma_px=(1.0, 3.0), keep_clean: bool = False) -> AlignmentSet:
    """Templates are blob sums at unit L2; images are moved templates + noise.

    snr is mean(clean^2) / noise_variance over the full frame; None gives
    noise-free images.  keep_clean also returns the noise-free images (the
    random stream, hence every other output, is unchanged).
    """
    rng = np.random.default_rng(seed)
    tb, temps, scales = [], [], []
    for _ in range(n_templates):
        b = random_blobs(rng, nblob, disk_px, sigma_px)
        img = render(b, n)
        sc = unit_l2_scale(img)
        b.amps = b.amps * sc
        tb.append(b)
        temps.append(img * sc)
        scales.append(sc)
    ib, imgs, cleans = [], [], []
    tt = np.zeros(n_images, dtype=np.int64)
    th = np.zeros(n_images)
    sh = np.zeros((n_images, 2))
    ns = np.zeros(n_images)
    for a in range(n_images):
        t = int(rng.integers(n_templates))
        theta = 2.0 * math.pi * rng.random()
        s = area_uniform_disk(rng, shift_radius_px)
        mb = tb[t].moved(theta, s)
        clean = render(mb, n)
        if snr is not None:
            sig = math.sqrt(float(np.mean(clean * clean)) / snr)
            noisy = clean + sig * rng.standard_normal((n, n))
        else:
            sig = 0.0
            noisy = clean
        tt[a], th[a], sh[a], ns[a] = t, theta, s, sig
        ib.append(mb)
        if keep_clean:
            cleans.append(clean)
        imgs.append(noisy)
    return AlignmentSet(n, np.array(temps), np.array(imgs), tb, ib,
                        np.array(scales), tt, th, sh, ns, np.array(cleans) if keep_clean else None)


def white_noise_images(seed: int, count: int, n: int) -> np.ndarray:
    """i.i.d. standard normal pixel images (worst case for band limits)."""
    return np.random.default_rng(seed).standard_normal((count, n, n))


# Named workloads -------------------------------------------------------------

#: The five workload shapes: images x templates, pixels, radial nodes M,
#: angular samples Qa (= number of rotations), shift radius R in pixels,
#: blobs per template, SNR, eps.
WORKLOADS = {
    "plain_n32": dict(n_images=4, n_templates=8, n=32, M=16, Qa=64, R=2.0,
                      nblob=20, snr=0.1, eps=1e-3),
    "cryoem_n128": dict(n_images=512, n_templates=2048, n=128, M=64, Qa=256,
                        R=4.0, nblob=60, snr=0.05, eps=1e-3),
}


def workload_set(name: str, seed: int, n_images: int | None = None,
                 n_templates: int | None = None) -> AlignmentSet:
    w = WORKLOADS[name]
    return make_alignment_set(seed, w["n"],
                              w["n_templates"] if n_templates is None else n_templates,
                              w["n_images"] if n_images is None else n_images,
                              w["nblob"], w["R"], w["snr"])


def ragged_stack_specs(seed: int, count: int = 64, scale: float = 1.0):
    """Per-stack shapes of the ragged batch workload.

    n ~ U{64, 96, 128, 192}; templates = round(exp(U[ln 100, ln 4000]));
    images ~ U{16..256}; shift radius ~ U{2, 2.5, ..., 8} px; M = n/2,
    Qa = 2n.  `scale` (< 1) shrinks image and template counts for tests.
    """
    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(count):
        n = int(rng.choice([64, 96, 128, 192]))
        nB = int(round(math.exp(rng.uniform(math.log(100), math.log(4000)))))
        nA = int(rng.integers(16, 257))
        R = 2.0 + 0.5 * int(rng.integers(0, 13))
        specs.append(dict(n=n, M=n // 2, Qa=2 * n, R=R,
                          n_templates=max(1, int(round(nB * scale))),
                          n_images=max(1, int(round(nA * scale)))))
    return specs


def mlp_init(seed: int, dims) -> list:
    """Initial MLP parameters [(W [out, in], b [out])], float32: He-normal
    weights (std sqrt(2 / fan_in)) for the ReLU layers, std sqrt(1 / fan_in)
    for the last (linear) layer, zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for i in range(len(dims) - 1):
        gain = 2.0 if i < len(dims) - 2 else 1.0
        W = rng.standard_normal((dims[i + 1], dims[i])) * math.sqrt(gain / dims[i])
        params.append((W.astype(np.float32), np.zeros(dims[i + 1], np.float32)))
    return params


def permutation(seed: int, n: int) -> np.ndarray:
    """A seeded random permutation of 0..n-1 (int32), e.g. minibatch order."""
    return np.random.default_rng(seed).permutation(n).astype(np.int32)


def gaussian_noise(seed: int, sigmas, n: int, device="cuda"):
    """Fresh white noise for re-noising clean images on the device:
    sigmas[i] * N(0, 1) per pixel, shape (len(sigmas), n, n), float32, from
    a seeded torch generator on `device`."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    sig = torch.as_tensor(np.asarray(sigmas, dtype=np.float32), device=device)
    z = torch.randn((sig.shape[0], n, n), generator=g, device=device, dtype=torch.float32)
    return z * sig[:, None, None]


def blob_power_spectrum(nterms: int = 16, sigma_lo_px: float = 1.0, sigma_hi_px: float = 3.0):
    """Expected radial power spectrum of the blob templates as a sum of
    Gaussians in y = k / Kmax (Kmax = pi n / 2): returns (alpha, beta) with
    P(y) = sum_j alpha_j exp(-beta_j y^2).

    A Gaussian blob of width s pixels (s dx in the image's units, dx = 2/n)
    has power exp(-k^2 s^2 dx^2) = exp(-pi^2 y^2 s^2) at radius k; blob
    centres are independent, so the cross terms average out and the power is
    the mean of that over s ~ U[sigma_lo, sigma_hi], here by the
    nterms-point Gauss-Legendre rule in s.  It does not depend on n.  A
    description of the input distribution, passed to the planner as a
    k-side weight."""
    x, wx = np.polynomial.legendre.leggauss(nterms)
    s = sigma_lo_px + (x + 1.0) * 0.5 * (sigma_hi_px - sigma_lo_px)
    return 0.5 * wx, (math.pi ** 2) * s ** 2
