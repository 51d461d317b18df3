"""Seeded synthetic inputs for the RTG-GMRES restoration problems.

This module only draws and lays out inputs: ground-truth images and videos,
the point-spread-function (PSF) band arrays, the random sketch matrices and the
direction of the additive noise.  It performs none of the solver's arithmetic
(no operator application, no sketching, no orthogonalisation); the blurred
observation C is formed by whoever consumes these inputs.

Conventions
-----------
* Tensors are numpy arrays indexed in the paper's order ``X[i1, i2, j]``
  (shape ``(I1, I2, J)``).  The device layout is column-major with ``i1``
  fastest, i.e. a C-contiguous array of shape ``(J, I2, I1)``;
  :func:`to_device_layout` / :func:`from_device_layout` convert.
* A banded factor ``M`` of size ``I x I`` with half-bandwidth ``r`` is stored
  row-major as ``band[i, d + r] = M[i, i + d]`` for ``-r <= d <= r`` (entries
  whose column falls outside ``[0, I)`` are zero: zero boundary conditions,
  Sec. 5.1).
* Canonical inputs are generated in float64 and rounded once to float32; both
  the GPU path and the oracle consume those float32 values.

Problem model (Sec. 5, eqs. (56)-(59)): C = A *_2 X *_1 B + N with a separable
Gaussian PSF (eq. (58)) on the two spatial modes, a channel/time mixing matrix
B on the third mode, and Gaussian noise N of relative level nu.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
from scipy import ndimage

F32 = np.float32


# --------------------------------------------------------------------------
# seeds
# --------------------------------------------------------------------------
def streams(seed: int, n_children: int = 0):
    """Independent generators for {image, noise, omega, aux} (+ children).

    Every config uses ``numpy.random.SeedSequence(seed).spawn``; batched
    configs spawn one child sequence per problem from the ``aux`` stream.
    """
    ss = np.random.SeedSequence(seed)
    image, noise, omega, aux = ss.spawn(4)
    out = {
        "image": np.random.default_rng(image),
        "noise": np.random.default_rng(noise),
        "omega": np.random.default_rng(omega),
        "aux": np.random.default_rng(aux),
    }
    if n_children:
        out["children"] = aux.spawn(n_children)
    return out


# --------------------------------------------------------------------------
# layout helpers
# --------------------------------------------------------------------------
def to_device_layout(x: np.ndarray) -> np.ndarray:
    """(I1, I2, J) paper-indexed array -> C-contiguous (J, I2, I1)."""
    return np.ascontiguousarray(np.asarray(x).transpose(2, 1, 0))


def from_device_layout(x: np.ndarray) -> np.ndarray:
    """C-contiguous (J, I2, I1) array -> (I1, I2, J) paper-indexed view."""
    return np.asarray(x).transpose(2, 1, 0)


# --------------------------------------------------------------------------
# images and videos
# --------------------------------------------------------------------------
def rectangles(rng, I1: int, I2: int, J: int, n_rect: int) -> np.ndarray:
    """Sum of axis-aligned rectangles with U(0,1) intensity per channel.

    Side lengths are uniform integers in [ceil(I/32), ceil(I/4)] per mode, the
    top-left corner is uniform inside the frame (rectangles are clipped at the
    border) and overlapping rectangles add.
    """
    x = np.zeros((I1, I2, J))
    lo1, hi1 = math.ceil(I1 / 32), max(math.ceil(I1 / 4), math.ceil(I1 / 32))
    lo2, hi2 = math.ceil(I2 / 32), max(math.ceil(I2 / 4), math.ceil(I2 / 32))
    for _ in range(n_rect):
        s1 = int(rng.integers(lo1, hi1 + 1))
        s2 = int(rng.integers(lo2, hi2 + 1))
        a1 = int(rng.integers(0, I1))
        a2 = int(rng.integers(0, I2))
        val = rng.uniform(0.0, 1.0, size=J)
        x[a1:a1 + s1, a2:a2 + s2, :] += val
    return x


def gaussian_random_field(rng, I1: int, I2: int, J: int, length: float = 16.0,
                          std: float = 0.2) -> np.ndarray:
    """White noise per channel smoothed by a Gaussian of std ``length`` pixels
    (periodic wrap), normalised to zero mean and standard deviation ``std``."""
    out = np.empty((I1, I2, J))
    for j in range(J):
        w = rng.standard_normal((I1, I2))
        f = ndimage.gaussian_filter(w, sigma=length, mode="wrap")
        f = f - f.mean()
        sd = f.std()
        out[:, :, j] = f * (std / sd if sd > 0 else 0.0)
    return out


def moving_rectangles_video(rng, I1: int, I2: int, T: int, n_rect: int = 20,
                            max_speed: float = 3.0) -> np.ndarray:
    """Grayscale video X[i1, i2, t]: rectangles moving at a constant random
    velocity (speed U(0, max_speed) px/frame, direction U(0, 2 pi)); the corner
    is rounded half-to-even each frame and the rectangle clipped to the frame."""
    x = np.zeros((I1, I2, T))
    lo1, hi1 = math.ceil(I1 / 32), math.ceil(I1 / 4)
    lo2, hi2 = math.ceil(I2 / 32), math.ceil(I2 / 4)
    for _ in range(n_rect):
        s1 = int(rng.integers(lo1, hi1 + 1))
        s2 = int(rng.integers(lo2, hi2 + 1))
        p1 = rng.uniform(0, I1)
        p2 = rng.uniform(0, I2)
        speed = rng.uniform(0.0, max_speed)
        ang = rng.uniform(0.0, 2 * math.pi)
        v1, v2 = speed * math.cos(ang), speed * math.sin(ang)
        val = rng.uniform(0.0, 1.0)
        for t in range(T):
            a1 = int(np.round(p1 + v1 * t))
            a2 = int(np.round(p2 + v2 * t))
            b1, e1 = max(a1, 0), min(a1 + s1, I1)
            b2, e2 = max(a2, 0), min(a2 + s2, I2)
            if b1 < e1 and b2 < e2:
                x[b1:e1, b2:e2, t] += val
    return x


# --------------------------------------------------------------------------
# operator factors (problem definition, Sec. 5.1-5.2)
# --------------------------------------------------------------------------
def gaussian_taps(sigma: float, r: int) -> np.ndarray:
    """1-D Gaussian PSF taps g[d], |d| <= r (eq. (58) is separable), normalised
    to sum 1 over the truncated support."""
    d = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-0.5 * (d / sigma) ** 2)
    return g / g.sum()


def half_bandwidth(sigma: float) -> int:
    """r = round-half-to-even(3 sigma): sigma 1.5 -> 4, 2 -> 6, 2.5 -> 8."""
    return int(np.round(3.0 * sigma))


def toeplitz_band(I: int, taps: np.ndarray) -> np.ndarray:
    """Band array of the zero-boundary convolution matrix M[i, k] = taps[i - k]
    (taps indexed -r..r), i.e. band[i, d + r] = M[i, i + d] = taps[-d]."""
    r = (len(taps) - 1) // 2
    band = np.zeros((I, 2 * r + 1))
    for d in range(-r, r + 1):
        lo, hi = max(0, -d), min(I, I - d)
        band[lo:hi, d + r] = taps[-d + r]
    return band


def gaussian_band(I: int, sigma: float, r: Optional[int] = None) -> np.ndarray:
    if r is None:
        r = half_bandwidth(sigma)
    return toeplitz_band(I, gaussian_taps(sigma, r))


def dense_to_band(M: np.ndarray, r: int) -> np.ndarray:
    """Band array of an arbitrary square matrix whose entries vanish outside
    the half-bandwidth r (used for the small channel-mixing matrix B)."""
    I = M.shape[0]
    band = np.zeros((I, 2 * r + 1))
    for i in range(I):
        for d in range(-r, r + 1):
            k = i + d
            if 0 <= k < I:
                band[i, d + r] = M[i, k]
    return band


def channel_mix(J: int = 3, diag: float = 0.7, off: float = 0.15) -> np.ndarray:
    """Cross-channel mixing matrix: ``diag`` on the diagonal, ``off`` elsewhere."""
    return np.full((J, J), off) + (diag - off) * np.eye(J)


def box_band(J: int, width: int = 5) -> np.ndarray:
    """Temporal motion blur: zero-boundary box filter of odd ``width``."""
    r = (width - 1) // 2
    return toeplitz_band(J, np.full(width, 1.0 / width))


def sketch_matrix(rng, l: int, I: int) -> Optional[np.ndarray]:
    """Mode-wise Gaussian sketch Omega in R^{l x I}, i.i.d. N(0, 1/l) so that
    E[Omega^T Omega] = I.  ``None`` (identity) when l == I."""
    if l == I:
        return None
    return rng.standard_normal((l, I)) / math.sqrt(l)


# --------------------------------------------------------------------------
# problem bundle
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    """All float32 canonical inputs of one restoration problem."""
    name: str
    x_true: np.ndarray          # (I1, I2, J) float32
    a1_band: np.ndarray         # (I1, 2 r1 + 1) float32
    a2_band: np.ndarray         # (I2, 2 r2 + 1) float32
    b_band: np.ndarray          # (J, 2 rB + 1) float32, band of B (C = ... *_1 B)
    om1: Optional[np.ndarray]   # (l1, I1) float32 or None (identity)
    om2: Optional[np.ndarray]   # (l2, I2)
    om3: Optional[np.ndarray]   # (l3, J)
    noise_dir: np.ndarray       # (I1, I2, J) float32, i.i.d. N(0, 1)
    nu: float                   # relative noise level ||N|| / ||A*X||
    m: int                      # Arnoldi steps
    sigma: float = 0.0

    @property
    def dims(self):
        return self.x_true.shape

    @property
    def r1(self):
        return (self.a1_band.shape[1] - 1) // 2

    @property
    def r2(self):
        return (self.a2_band.shape[1] - 1) // 2

    @property
    def rB(self):
        return (self.b_band.shape[1] - 1) // 2

    @property
    def sketch_dims(self):
        I1, I2, J = self.dims
        return (I1 if self.om1 is None else self.om1.shape[0],
                I2 if self.om2 is None else self.om2.shape[0],
                J if self.om3 is None else self.om3.shape[0])


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=F32)


def make_image_problem(name, seed, I1, I2, n_rect, grf, sigma, r, nu, l1, l2, m,
                       J=3, rng_set=None) -> Problem:
    rs = rng_set if rng_set is not None else streams(seed)
    x = rectangles(rs["image"], I1, I2, J, n_rect)
    if grf:
        x = x + gaussian_random_field(rs["image"], I1, I2, J)
    B = channel_mix(J)
    return Problem(
        name=name,
        x_true=_f32(x),
        a1_band=_f32(gaussian_band(I1, sigma, r)),
        a2_band=_f32(gaussian_band(I2, sigma, r)),
        b_band=_f32(dense_to_band(B, J - 1)),
        om1=_f32(sketch_matrix(rs["omega"], l1, I1)),
        om2=_f32(sketch_matrix(rs["omega"], l2, I2)),
        om3=None,
        noise_dir=_f32(rs["noise"].standard_normal((I1, I2, J))),
        nu=float(nu), m=int(m), sigma=float(sigma),
    )


def rotated_gaussian_psf(r: int, s_major: float, s_minor: float, theta: float) -> np.ndarray:
    """Non-separable PSF of size (2r+1) x (2r+1): an anisotropic Gaussian
    whose axes are rotated by theta (a general PSF P of eq. (57); row index
    along i1, column index along i2, centre at [r, r]), normalised to sum 1.
    For theta not a multiple of pi/2 and unequal widths it is not an outer
    product of two tap vectors."""
    d = np.arange(-r, r + 1, dtype=np.float64)
    a, b = np.meshgrid(d, d, indexing="ij")
    c, s = math.cos(theta), math.sin(theta)
    u = c * a + s * b
    v = -s * a + c * b
    P = np.exp(-0.5 * (u / s_major) ** 2 - 0.5 * (v / s_minor) ** 2)
    return P / P.sum()


@dataclasses.dataclass
class PSFProblem:
    """Canonical float32 inputs of a restoration problem with a general
    (non-separable) PSF applied to every channel, then the channel mix B."""
    name: str
    x_true: np.ndarray          # (I1, I2, J) float32
    psf: np.ndarray             # (2r+1, 2r+1) float32, orientation of eq. (57)
    b_band: np.ndarray          # (J, 2 rB + 1) float32
    om1: Optional[np.ndarray]
    om2: Optional[np.ndarray]
    om3: Optional[np.ndarray]
    noise_dir: np.ndarray
    nu: float
    m: int

    @property
    def dims(self):
        return self.x_true.shape

    @property
    def r(self):
        return (self.psf.shape[0] - 1) // 2

    @property
    def rB(self):
        return (self.b_band.shape[1] - 1) // 2


def psf_problem(seed: int, I1: int, I2: int, J: int = 3, r: int = 4, l1: int = 16, l2: int = 16,
                l3: Optional[int] = None, m: int = 20, nu: float = 1e-2, n_rect: int = 20,
                grf: bool = False, s_major: float = 2.0, s_minor: float = 0.8,
                theta: float = 0.6) -> PSFProblem:
    """Rectangles (+ optional Gaussian random field) blurred by a rotated
    anisotropic Gaussian PSF of radius r, the 3x3-style channel mix (or a
    random band for J != 3), Gaussian sketches (Om3 only when l3 < J)."""
    rs = streams(seed)
    x = rectangles(rs["image"], I1, I2, J, n_rect)
    if grf:
        x = x + gaussian_random_field(rs["image"], I1, I2, J)
    if J == 3:
        b_band = dense_to_band(channel_mix(3), 2)
    else:
        b_band = rs["aux"].uniform(0.05, 0.3, (J, 3))
        b_band[:, 1] += 0.5
        b_band[0, 0] = 0.0
        b_band[-1, 2] = 0.0
    l3v = J if l3 is None else l3
    return PSFProblem(
        name=f"psf_{I1}x{I2}x{J}_r{r}",
        x_true=_f32(x),
        psf=_f32(rotated_gaussian_psf(r, s_major, s_minor, theta)),
        b_band=_f32(b_band),
        om1=_f32(sketch_matrix(rs["omega"], l1, I1)),
        om2=_f32(sketch_matrix(rs["omega"], l2, I2)),
        om3=_f32(sketch_matrix(rs["omega"], l3v, J)) if l3v < J else None,
        noise_dir=_f32(rs["noise"].standard_normal((I1, I2, J))),
        nu=float(nu), m=int(m),
    )


def cfg2_psf(seed: int = 0) -> PSFProblem:
    """512x512x3 like cfg2, blurred by a 9x9 rotated anisotropic Gaussian
    PSF (widths 2.0 and 0.8 px, axes at 0.6 rad): a non-separable blur."""
    return psf_problem(seed, 512, 512, 3, r=4, l1=64, l2=64, m=50, nu=1e-3, n_rect=200, grf=True)


def cfg1(seed: int = 0) -> Problem:
    """32x32x3 colour image, 20 rectangles; sigma 1.5, r 4; nu 1e-2;
    sketch 16x16x3; m = 20."""
    return make_image_problem("cfg1_32x32x3", seed, 32, 32, 20, False, 1.5, 4,
                              1e-2, 16, 16, 20)


def cfg2(seed: int = 0) -> Problem:
    """512x512x3 colour image, 200 rectangles + Gaussian random field;
    sigma 2.5, r 8; nu 1e-3; sketch 64x64x3; m = 50."""
    return make_image_problem("cfg2_512x512x3", seed, 512, 512, 200, True, 2.5,
                              8, 1e-3, 64, 64, 50)


def cfg3(seed: int = 0) -> Problem:
    """256x256x64 grayscale video of moving rectangles; spatial sigma 2, r 6;
    temporal box blur of width 5; nu 1e-3; sketch 48x48x16; m = 80."""
    rs = streams(seed)
    x = moving_rectangles_video(rs["image"], 256, 256, 64)
    return Problem(
        name="cfg3_video_256x256x64",
        x_true=_f32(x),
        a1_band=_f32(gaussian_band(256, 2.0, 6)),
        a2_band=_f32(gaussian_band(256, 2.0, 6)),
        b_band=_f32(box_band(64, 5)),
        om1=_f32(sketch_matrix(rs["omega"], 48, 256)),
        om2=_f32(sketch_matrix(rs["omega"], 48, 256)),
        om3=_f32(sketch_matrix(rs["omega"], 16, 64)),
        noise_dir=_f32(rs["noise"].standard_normal((256, 256, 64))),
        nu=1e-3, m=80, sigma=2.0,
    )


def _round16(v: float) -> int:
    """Round half-up to a multiple of 16."""
    return int(math.floor(v / 16.0 + 0.5)) * 16


def _child_streams(seed: int, p: int):
    """Streams of problem p of a batched config: child p of the aux stream of
    SeedSequence(seed) (spawn key (3, p)), re-seeded from its first word."""
    child = np.random.SeedSequence(seed, spawn_key=(3, p))
    return streams(int(child.generate_state(1)[0]))


def cfg4_problem(seed: int, p: int, m: int = 40) -> Problem:
    """Problem p of the uneven batch: sides uniform integers in [64, 512]
    rounded to multiples of 16, sigma ~ U(1,3) (r = round-half-even(3 sigma)),
    nu ~ U[1e-3, 1e-2], sketch sides I/4 (channel mode identity)."""
    cr = _child_streams(seed, p)
    aux = cr["aux"]
    I1 = _round16(aux.integers(64, 513))
    I2 = _round16(aux.integers(64, 513))
    sigma = float(aux.uniform(1.0, 3.0))
    nu = float(aux.uniform(1e-3, 1e-2))
    return make_image_problem(f"cfg4_{p}", 0, I1, I2, 200, True, sigma, half_bandwidth(sigma), nu,
                              I1 // 4, I2 // 4, m, rng_set=cr)


def cfg4(seed: int = 0, count: int = 256, m: int = 40):
    """Batch of ``count`` independent colour images of uneven size, m = 40."""
    return [cfg4_problem(seed, p, m) for p in range(count)]


def cfg5_problem(seed: int, p: int, side: int = 128, m: int = 50) -> Problem:
    """Training problem p for the learned warm start: the cfg2 generator at
    side x side x 3 (200 rectangles + Gaussian random field), sigma ~ U(1,3),
    nu ~ U[1e-3, 1e-2]; label solver sketch I/8 per spatial mode, m = 50."""
    cr = _child_streams(seed, p)
    aux = cr["aux"]
    sigma = float(aux.uniform(1.0, 3.0))
    nu = float(aux.uniform(1e-3, 1e-2))
    return make_image_problem(f"cfg5_{p}", 0, side, side, 200, True, sigma, half_bandwidth(sigma),
                              nu, side // 8, side // 8, m, rng_set=cr)


def cfg5_train(seed: int = 0, count: int = 20000, side: int = 128, m: int = 50):
    for p in range(count):
        yield cfg5_problem(seed, p, side, m)


def small_problem(seed: int, I1: int, I2: int, J: int, r1: int, r2: int,
                  rB: int, l1: int, l2: int, l3: int, m: int,
                  nu: float = 1e-2, symmetric_b: bool = False,
                  random_bands: bool = False) -> Problem:
    """Small problems of arbitrary shape for parity and edge-case tests.

    ``random_bands`` draws non-symmetric band entries (so that transposition
    and orientation mistakes change the result); otherwise Gaussian bands.
    """
    rs = streams(seed)
    rng = rs["aux"]
    x = rectangles(rs["image"], I1, I2, J, 6) + 0.1 * rs["image"].standard_normal((I1, I2, J))
    if random_bands:
        a1 = toeplitz_band(I1, rng.uniform(0.1, 1.0, 2 * r1 + 1))
        a1 = a1 * rng.uniform(0.8, 1.2, size=(I1, 1))
        a2 = toeplitz_band(I2, rng.uniform(0.1, 1.0, 2 * r2 + 1))
        bm = rng.uniform(0.1, 1.0, size=(J, J))
        bm = np.triu(np.tril(bm, rB), -rB)
    else:
        a1 = gaussian_band(I1, max(r1, 1) / 3.0, r1)
        a2 = gaussian_band(I2, max(r2, 1) / 3.0, r2)
        bm = channel_mix(J) if J > 1 else np.eye(1)
        bm = np.triu(np.tril(bm, rB), -rB)
    if symmetric_b:
        bm = 0.5 * (bm + bm.T)
    return Problem(
        name=f"small_{I1}x{I2}x{J}",
        x_true=_f32(x),
        a1_band=_f32(a1), a2_band=_f32(a2),
        b_band=_f32(dense_to_band(bm, rB)),
        om1=_f32(sketch_matrix(rs["omega"], l1, I1)),
        om2=_f32(sketch_matrix(rs["omega"], l2, I2)),
        om3=_f32(sketch_matrix(rs["omega"], l3, J)),
        noise_dir=_f32(rs["noise"].standard_normal((I1, I2, J))),
        nu=float(nu), m=int(m),
    )


CONFIGS = {"cfg1": cfg1, "cfg2": cfg2, "cfg3": cfg3}
