"""Seeded synthetic inputs for the matrix equation AXB = C.

This module only *builds problem instances*: it draws A, B and X* from a
seeded generator and forms the consistent right-hand side C = A X* B (or a
noisy one). It contains none of the solver's arithmetic, and both the CPU
oracle and the GPU path take their inputs from here.

Sources of the shapes and distributions:
  * Section 5 of the paper draws X with randn(p, q), takes dense A, B with
    iid N(0,1) entries, and sets C = A X B so the system is consistent.
  * Example 5.2 builds rank-deficient pairs by stacking copies of a random
    matrix, e.g. [A, A] and [B; B] (Tables 5 and 7).
  * Section 6 restores blurred colour images; the separable Toeplitz-blur
    stand-in below (per-channel A X B with A, B banded Gaussian blurs) is a
    synthetic substitute, because the paper's test images are not available.

All arrays are float64, C-contiguous, row-major. Every generator is a pure
function of its seed (numpy PCG64 via default_rng), drawn in the order the
docstring states, so the same call always gives the same bytes.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Instance:
    """One problem AXB = C plus the data used to judge a solution.

    A: m x p, B: q x n, C: m x n, X_star: p x q (the generating solution, or
    None when C is not consistent with a known X). X0 is the initial guess
    (None means zero). `name` describes the recipe.
    """

    name: str
    A: np.ndarray
    B: np.ndarray
    C: np.ndarray
    X_star: Optional[np.ndarray]
    X0: Optional[np.ndarray] = None

    @property
    def shape(self):
        m, p = self.A.shape
        q, n = self.B.shape
        return m, p, q, n


def _c(x: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float64)


def gaussian_consistent(m: int, p: int, q: int, n: int, seed: int,
                        name: str = "") -> Instance:
    """A (m x p), B (q x n), X* (p x q) iid N(0,1), drawn in that order; C = A X* B."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, p))
    B = rng.standard_normal((q, n))
    X = rng.standard_normal((p, q))
    C = A @ X @ B
    return Instance(name or f"randn m={m} p={p} q={q} n={n} seed={seed}",
                    _c(A), _c(B), _c(C), _c(X))


def rank_deficient_left(m: int, p: int, q: int, n: int, rank: int, seed: int,
                        name: str = "") -> Instance:
    """A = U V with U (m x rank), V (rank x p); B (q x n), X* (p x q) iid N(0,1).

    Draw order: U, V, B, X*. C = A X* B is consistent; the least-norm
    solution is A^+ C B^+, which differs from X* because A is rank deficient.
    """
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((m, rank))
    V = rng.standard_normal((rank, p))
    B = rng.standard_normal((q, n))
    X = rng.standard_normal((p, q))
    A = U @ V
    C = A @ X @ B
    return Instance(name or f"rankdef m={m} p={p} r={rank} q={q} n={n} seed={seed}",
                    _c(A), _c(B), _c(C), _c(X))


def stacked_rank_deficient(m: int, p: int, q: int, n: int, seed: int,
                           a_mode: str = "cols", b_mode: str = "rows",
                           name: str = "") -> Instance:
    """Rank-deficient pair built by duplication, as in the paper's Tables 5/7.

    a_mode "cols": A = [A0, A0] with A0 (m x p/2); "rows": A = [A0; A0] with
    A0 (m/2 x p). b_mode "rows": B = [B0; B0] with B0 (q/2 x n); "cols":
    B = [B0, B0] with B0 (q x n/2). Draw order: A0, B0, X*.
    """
    rng = np.random.default_rng(seed)
    if a_mode == "cols":
        A0 = rng.standard_normal((m, p // 2))
        A_parts = (A0, A0)
        A_stack = np.hstack
    else:
        A0 = rng.standard_normal((m // 2, p))
        A_parts = (A0, A0)
        A_stack = np.vstack
    if b_mode == "rows":
        B0 = rng.standard_normal((q // 2, n))
        B = np.vstack((B0, B0))
    else:
        B0 = rng.standard_normal((q, n // 2))
        B = np.hstack((B0, B0))
    A = A_stack(A_parts)
    X = rng.standard_normal((A.shape[1], B.shape[0]))
    C = A @ X @ B
    return Instance(name or f"stacked {a_mode}/{b_mode} seed={seed}",
                    _c(A), _c(B), _c(C), _c(X))


def with_zero_rows(inst: Instance, rows) -> Instance:
    """Copy of `inst` with the given rows of A (and of C) set to zero.

    Zero rows of A make the corresponding subsystems A_i X B = C_i void; the
    solver must skip them (their weight ||A_i||^2 is zero).
    """
    A = inst.A.copy()
    C = inst.C.copy()
    A[list(rows), :] = 0.0
    C[list(rows), :] = 0.0
    return Instance(inst.name + f" zero-rows={list(rows)}", _c(A), _c(inst.B),
                    _c(C), None if inst.X_star is None else inst.X_star.copy())


def shared_ab_batch(inst: Instance, nb: int, seed: int):
    """nb consistent instances sharing inst's A and B: X*_b iid N(0,1) drawn
    in order b = 0..nb-1 from default_rng(seed), C_b = A X*_b B."""
    rng = np.random.default_rng(seed)
    p, q = inst.A.shape[1], inst.B.shape[0]
    out = []
    for b in range(nb):
        X = rng.standard_normal((p, q))
        out.append(Instance(inst.name + f" batch {b}/{nb} seed={seed}", inst.A, inst.B,
                            _c(inst.A @ X @ inst.B), _c(X)))
    return out


def ragged_batch(nb: int, seed: int, mn_range=(128, 1024), pq_range=(64, 512)):
    """Independent consistent instances of uneven size: first all sizes, m and
    n uniform on the integers of mn_range, p and q on pq_range (inclusive),
    in the order (m, p, q, n) per instance; then A (m x p), B (q x n),
    X* (p x q) iid N(0,1) per instance in order, all from default_rng(seed);
    C_b = A_b X*_b B_b."""
    rng = np.random.default_rng(seed)
    sizes = []
    for _ in range(nb):
        m = int(rng.integers(mn_range[0], mn_range[1] + 1))
        p = int(rng.integers(pq_range[0], pq_range[1] + 1))
        q = int(rng.integers(pq_range[0], pq_range[1] + 1))
        n = int(rng.integers(mn_range[0], mn_range[1] + 1))
        sizes.append((m, p, q, n))
    out = []
    for b, (m, p, q, n) in enumerate(sizes):
        A = rng.standard_normal((m, p))
        B = rng.standard_normal((q, n))
        X = rng.standard_normal((p, q))
        out.append(Instance(f"ragged batch seed={seed} #{b} m={m} p={p} q={q} n={n}",
                            _c(A), _c(B), _c(A @ X @ B), _c(X)))
    return out


def blur_toeplitz(size: int, sigma: float, half_width: int = 4) -> np.ndarray:
    """Banded Toeplitz Gaussian blur (2*half_width+1 taps), each row divided by its sum.

    Tap weight exp(-d^2 / (2 sigma^2)) for |d| <= half_width; rows at the
    border lose the taps that fall outside and are renormalised to sum 1.
    """
    i = np.arange(size)
    d = i[:, None] - i[None, :]
    K = np.where(np.abs(d) <= half_width, np.exp(-(d.astype(np.float64) ** 2) / (2.0 * sigma ** 2)), 0.0)
    K /= K.sum(axis=1, keepdims=True)
    return _c(K)


def banded_gaussian(size: int, seed: int, sigma: float = 2.0, half_width: int = 4) -> Instance:
    """The blur pair A = blur_toeplitz(size, sigma, half_width), B = A^T with
    X* iid N(0,1) from default_rng(seed) (no flat regions, so no ties in the
    greedy ratios) and C = A X* B."""
    A = blur_toeplitz(size, sigma, half_width)
    B = _c(A.T)
    X = np.random.default_rng(seed).standard_normal((size, size))
    return Instance(f"banded gaussian size={size} sigma={sigma} seed={seed}", A, B, _c(A @ X @ B),
                    _c(X))


def sparse_random(m: int, p: int, q: int, n: int, seed: int, row_nnz=(2, 4),
                  col_nnz=(1, 3), empty_rows: int = 0) -> Instance:
    """Irregular sparse A (m x p): each row holds a number of N(0,1) entries
    drawn uniformly from row_nnz (inclusive) at distinct random columns,
    then `empty_rows` distinct random rows are cleared. B (q x n): each
    column holds col_nnz entries at distinct random rows. X* iid N(0,1);
    C = A X* B. All from default_rng(seed) in that order. With at least two
    entries per row, no two rows of A are parallel (parallel rows have equal
    ratios ||R_i||^2 / ||A_i||^2 at every update, an exact tie)."""
    rng = np.random.default_rng(seed)
    A = np.zeros((m, p))
    for i in range(m):
        k = int(rng.integers(row_nnz[0], row_nnz[1] + 1))
        cols = rng.choice(p, size=k, replace=False)
        A[i, cols] = rng.standard_normal(k)
    if empty_rows:
        A[rng.choice(m, size=empty_rows, replace=False)] = 0.0
    B = np.zeros((q, n))
    for j in range(n):
        k = int(rng.integers(col_nnz[0], col_nnz[1] + 1))
        rows = rng.choice(q, size=k, replace=False)
        B[rows, j] = rng.standard_normal(k)
    X = rng.standard_normal((p, q))
    return Instance(f"sparse random m={m} p={p} q={q} n={n} seed={seed}", _c(A), _c(B),
                    _c(A @ X @ B), _c(X))


def gaussian_taps(size: int = 5, sigma: float = 6.0) -> np.ndarray:
    """The 1-D factor g of the size x size Gaussian kernel exp(-(x^2 + y^2) /
    (2 sigma^2)) normalised to sum 1: the 2-D kernel is the outer product
    g g^T (g itself sums to 1)."""
    x = np.arange(size) - (size - 1) / 2.0
    g = np.exp(-x ** 2 / (2.0 * sigma ** 2))
    return g / g.sum()


def blur_factor(n: int, taps: np.ndarray) -> np.ndarray:
    """n x n Toeplitz matrix applying the centred 1-D taps with zero
    padding (no renormalisation at the border)."""
    h = len(taps) // 2
    T = np.zeros((n, n))
    for i in range(n):
        for d in range(-h, h + 1):
            if 0 <= i + d < n:
                T[i, i + d] = taps[d + h]
    return T


# The cross-channel blurring matrix printed in the paper's colour image
# example (rows: output channel R, G, B).
CROSS_CHANNEL = np.array([[0.9, 0.05, 0.05], [0.0, 0.9, 0.1], [0.05, 0.1, 0.85]])


def paper_image_model(h: int, w: int, seed: int, size: int = 5, sigma: float = 6.0,
                      random_image: bool = False) -> Instance:
    """The paper's colour-image model A X A_c^T = C on a synthetic h x w x 3
    image: X (hw x 3) holds the column-major vectorised channels, A (hw x hw)
    = T_w kron T_h is the 2-D Gaussian blur (size x size taps, sigma, zero
    padding), B = A_c^T (3 x 3). Built densely (for the sizes of tests).
    random_image: X iid N(0,1) from default_rng(seed) instead of the
    synthetic picture (whose flat regions give rows with equal ratios, exact
    ties that rounding breaks differently in different summation orders)."""
    g = gaussian_taps(size, sigma)
    A = np.kron(blur_factor(w, g), blur_factor(h, g))
    if random_image:
        X = np.random.default_rng(seed).standard_normal((h * w, 3))
    else:
        img = synthetic_image(h, w, 3, seed)
        X = np.stack([img[c].T.reshape(-1) for c in range(3)], axis=1)
    B = CROSS_CHANNEL.T.copy()
    return Instance(f"paper image model {h}x{w} seed={seed}", _c(A), _c(B), _c(A @ X @ B), _c(X))


def synthetic_image(h: int, w: int, channels: int, seed: int,
                    n_rect: int = 8, n_disc: int = 8) -> np.ndarray:
    """channels x h x w image in [0,1]: a per-channel linear gradient, then
    axis-aligned rectangles and discs with shared geometry and per-channel
    intensity, painted in order and clipped to [0, 1].
    """
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    img = np.empty((channels, h, w))
    for c in range(channels):
        c0 = rng.uniform(0.0, 0.5)
        c1, c2 = rng.uniform(-0.25, 0.25, size=2)
        img[c] = c0 + c1 * xx / max(w - 1, 1) + c2 * yy / max(h - 1, 1)
    lo, hi = max(2, min(h, w) // 16), max(3, min(h, w) // 3)
    for _ in range(n_rect):
        rh, rw = rng.integers(lo, hi, size=2)
        y0 = rng.integers(0, max(1, h - rh))
        x0 = rng.integers(0, max(1, w - rw))
        val = rng.uniform(0.0, 1.0, size=channels)
        img[:, y0:y0 + rh, x0:x0 + rw] = val[:, None, None]
    for _ in range(n_disc):
        rad = rng.integers(max(1, lo // 2), max(2, hi // 2))
        cy, cx = rng.integers(0, h), rng.integers(0, w)
        mask = (yy - cy) ** 2 + (xx - cx) ** 2 <= rad ** 2
        val = rng.uniform(0.0, 1.0, size=channels)
        for c in range(channels):
            img[c][mask] = val[c]
    return np.clip(img, 0.0, 1.0)


def blurred_image(size: int, channels: int, sigma: float, seed: int,
                  noise_std: float = 0.0, half_width: int = 4):
    """Per-channel instances C_c = A X*_c B (+ noise) with A = blur, B = A^T.

    Returns a list of `channels` Instances sharing A and B. Noise is drawn
    after the image, from default_rng(seed + 1), iid N(0, noise_std^2).
    """
    A = blur_toeplitz(size, sigma, half_width)
    B = _c(A.T)
    img = synthetic_image(size, size, channels, seed)
    noise_rng = np.random.default_rng(seed + 1)
    out = []
    for c in range(channels):
        X = _c(img[c])
        C = A @ X @ B
        if noise_std > 0:
            C = C + noise_rng.standard_normal(C.shape) * noise_std
        out.append(Instance(f"blur size={size} sigma={sigma} ch={c} seed={seed}",
                            A, B, _c(C), X))
    return out


# --------------------------------------------------------------------------
# Named workloads.
#   small:   A 100x40, B 40x100, X* 40x40 iid N(0,1) (data seed 1).
#   large:   A 2000x500, B 500x2000, X* 500x500 iid N(0,1) (data seed 2).
#   large_rankdef: A = U(2000x250) V(250x500), B 500x2000 (data seed 3).
#   ragged:  a mid-size case whose rows and columns do not divide evenly
#            over work-groups (data seed 11).
# --------------------------------------------------------------------------

def warmstart_image(seed: int, size: int = 256, channels: int = 3, sigma_range=(1.0, 3.0),
                    half_width: int = 4):
    """One image of the learned-warm-start workload: sigma uniform on
    sigma_range from default_rng(seed), then the synthetic image of
    synthetic_image(seed + 1); A = blur_toeplitz(size, sigma), B = A^T,
    C_c = A X*_c B without noise. Returns (A, B, C (channels, size, size),
    X* (channels, size, size), sigma)."""
    sigma = float(np.random.default_rng(seed).uniform(*sigma_range))
    A = blur_toeplitz(size, sigma, half_width)
    B = _c(A.T)
    X = synthetic_image(size, size, channels, seed + 1)
    C = np.stack([A @ X[c] @ B for c in range(channels)])
    return A, B, _c(C), _c(X), sigma


def bf16_bits(x) -> np.ndarray:
    """BF16 bit patterns (uint16) of x rounded to nearest even (via FP32)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def bf16_values(bits) -> np.ndarray:
    """The float64 values of BF16 bit patterns."""
    return (np.asarray(bits, np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16_random(rng, shape, scale=1.0) -> np.ndarray:
    """N(0, scale^2) draws rounded to BF16 (float64 holding BF16 values)."""
    return bf16_values(bf16_bits(scale * rng.standard_normal(shape)))


def small(seed: int = 1) -> Instance:
    return gaussian_consistent(100, 40, 40, 100, seed, name="small 100x40 / 40x100")


def large(seed: int = 2) -> Instance:
    return gaussian_consistent(2000, 500, 500, 2000, seed, name="large 2000x500 / 500x2000")


def large_rankdef(seed: int = 3) -> Instance:
    return rank_deficient_left(2000, 500, 500, 2000, 250, seed,
                               name="large rank-250 A 2000x500 / 500x2000")


def ragged(seed: int = 11) -> Instance:
    return gaussian_consistent(333, 70, 52, 261, seed, name="ragged 333x70 / 52x261")


# The paper's randn-built sets (Example 5.2), regenerated in distribution.
def paper_table3_set2(trial: int) -> Instance:
    """Table 3 Set 2: A = randn(140, 30), B = randn(70, 160)."""
    return gaussian_consistent(140, 30, 70, 160, 7000 + trial, name="T3S2")


def paper_table3_set5(trial: int) -> Instance:
    """Table 3 Set 5: A = randn(230, 50), B = randn(110, 240)."""
    return gaussian_consistent(230, 50, 110, 240, 7100 + trial, name="T3S5")


def paper_table1_set2(trial: int) -> Instance:
    """Table 1 Set 2: A = randn(110, 45), B = randn(50, 140)."""
    return gaussian_consistent(110, 45, 50, 140, 7200 + trial, name="T1S2")
