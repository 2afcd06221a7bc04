"""Seeded generators for the solver workloads.

Every generator takes an integer seed and returns a :class:`Problem` whose
matrix is either a CSR (int32 row pointers and column indices, float64 values,
columns sorted and unique inside each row) or a dense row-major float64 array.
Right-hand sides are built as ``b = A @ x_star`` so the systems are consistent
unless stated otherwise.

Shapes follow the workloads the solvers are measured on:

* dense Gaussian square systems (i.i.d. N(0,1) entries);
* the 2-D convection-diffusion 5-point stencil, -Lap(u) + g (u_x + u_y), on the
  unit square with zero Dirichlet data and central differences (the PDE the
  paper's convection-diffusion experiment discretises, section 5.1.8);
* the Kac / Clement tridiagonal matrix (section 5.1.6 uses Clement matrices);
* an LP-shaped wide sparse matrix, m x n with n >> m, six nonzeros per column
  plus an identity slack block (the m = 1e4, n up to 1e6 class of section 5.3);
* batches of uneven Poisson stencils and diagonally dominant random sparse
  systems with several right-hand sides each;
* a randomly perturbed Poisson stencil;
* sparse matrices with heavy-tailed (Pareto) row lengths, optionally with
  empty rows and fully dense rows (the skewed operands the merge-path product
  is for).

No solver arithmetic lives here.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Distinct stream ids so that two workloads with the same seed do not share
# random numbers.
_STREAM = {
    "dense": 1,
    "convdiff": 2,
    "kac": 3,
    "lp": 4,
    "batched": 5,
    "stencil_perturbed": 6,
    "randsparse": 7,
    "skewed": 8,
}


def _rng(kind: str, seed: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), _STREAM[kind]])


@dataclasses.dataclass
class Csr:
    """Compressed sparse rows: ``row_ptr`` (m+1), ``col_idx`` (nnz), ``val`` (nnz)."""

    m: int
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self) -> np.ndarray:
        out = np.zeros((self.m, self.n), dtype=np.float64)
        rows = np.repeat(np.arange(self.m), np.diff(self.row_ptr))
        out[rows, self.col_idx] = self.val
        return out

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.m, self.n))

    def matvec(self, x: np.ndarray) -> np.ndarray:
        """Plain product used only to build right-hand sides."""
        return self.to_scipy() @ x


@dataclasses.dataclass
class Problem:
    name: str
    A: object  # Csr or np.ndarray (dense, row-major)
    b: np.ndarray
    x_star: Optional[np.ndarray] = None
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def dense(self) -> bool:
        return isinstance(self.A, np.ndarray)

    @property
    def shape(self):
        return (self.A.shape if self.dense else (self.A.m, self.A.n))


def csr_from_coo(m: int, n: int, rows, cols, vals) -> Csr:
    """Build a canonical CSR (sorted columns, duplicates summed)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    if rows.size:
        if rows.min() < 0 or rows.max() >= m or cols.min() < 0 or cols.max() >= n:
            raise ValueError("coordinate out of range")
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key, rows, cols, vals = key[order], rows[order], cols[order], vals[order]
    if rows.size:
        first = np.ones(key.size, dtype=bool)
        first[1:] = key[1:] != key[:-1]
        summed = vals[first]
        if not first.all():
            # Duplicates are summed in their coordinate order.
            grp = np.cumsum(first) - 1
            dup = ~first
            np.add.at(summed, grp[dup], vals[dup])
        rows, cols, vals = rows[first], cols[first], summed
    counts = np.bincount(rows, minlength=m) if rows.size else np.zeros(m, dtype=np.int64)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32")
    return Csr(m, n, row_ptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64))


def csr_from_dense(a: np.ndarray, keep_zeros: bool = False) -> Csr:
    a = np.asarray(a, dtype=np.float64)
    m, n = a.shape
    if keep_zeros:
        rows, cols = np.divmod(np.arange(m * n), n)
        return csr_from_coo(m, n, rows, cols, a.reshape(-1))
    rows, cols = np.nonzero(a)
    return csr_from_coo(m, n, rows, cols, a[rows, cols])


# --------------------------------------------------------------------------
# dense Gaussian
# --------------------------------------------------------------------------
def dense_gaussian(n: int = 500, seed: int = 0, m: Optional[int] = None) -> Problem:
    """A with i.i.d. N(0,1) entries (m x n, default square), x* ~ N(0,1), b = A x*."""
    m = n if m is None else m
    g = _rng("dense", seed)
    a = g.standard_normal((m, n))
    xs = g.standard_normal(n)
    b = a @ xs
    return Problem(f"dense_gaussian_{m}x{n}_s{seed}", np.ascontiguousarray(a), b, xs,
                   {"m": m, "n": n, "seed": seed})


# --------------------------------------------------------------------------
# 5-point stencils
# --------------------------------------------------------------------------
def _stencil5(nx: int, ny: int, c_diag, c_w, c_e, c_s, c_n) -> Csr:
    """5-point stencil on an nx x ny grid, lexicographic with x fastest."""
    idx = np.arange(nx * ny, dtype=np.int64)
    ix = idx % nx
    iy = idx // nx
    rows = [idx]
    cols = [idx]
    vals = [np.full(idx.size, c_diag, dtype=np.float64)]
    for mask, off, c in ((ix > 0, -1, c_w), (ix < nx - 1, 1, c_e),
                         (iy > 0, -nx, c_s), (iy < ny - 1, nx, c_n)):
        r = idx[mask]
        rows.append(r)
        cols.append(r + off)
        vals.append(np.full(r.size, c, dtype=np.float64))
    return csr_from_coo(nx * ny, nx * ny, np.concatenate(rows), np.concatenate(cols),
                        np.concatenate(vals))


def convection_diffusion(N: int = 512, gamma: float = 10.0, seed: int = 0) -> Problem:
    """-Lap(u) + gamma (u_x + u_y) on the unit square, N x N interior points.

    Central differences with h = 1/(N+1), scaled by h^2: diagonal 4, west and
    south -1 - gamma h / 2, east and north -1 + gamma h / 2.  x* ~ U[0,1].
    """
    h = 1.0 / (N + 1)
    A = _stencil5(N, N, 4.0, -1.0 - gamma * h / 2, -1.0 + gamma * h / 2,
                  -1.0 - gamma * h / 2, -1.0 + gamma * h / 2)
    xs = _rng("convdiff", seed).uniform(0.0, 1.0, A.n)
    return Problem(f"convdiff_{N}x{N}_g{gamma:g}_s{seed}", A, A.matvec(xs), xs,
                   {"N": N, "gamma": gamma, "seed": seed})


def poisson5(nx: int, ny: Optional[int] = None) -> Csr:
    """Poisson 5-point matrix (4 on the diagonal, -1 to each grid neighbour)."""
    ny = nx if ny is None else ny
    return _stencil5(nx, ny, 4.0, -1.0, -1.0, -1.0, -1.0)


def perturbed_stencil(N: int = 256, sigma: float = 0.1, seed: int = 0) -> Problem:
    """Poisson 5-point stencil with N(0, sigma) added to every stored nonzero."""
    A = poisson5(N)
    g = _rng("stencil_perturbed", seed)
    A.val = A.val + g.normal(0.0, sigma, A.nnz)
    xt = g.standard_normal(A.n)
    xs = g.standard_normal(A.n)
    return Problem(f"stencil_perturbed_{N}x{N}_s{seed}", A, A.matvec(xs), xs,
                   {"N": N, "sigma": sigma, "seed": seed, "x_target": xt})


# --------------------------------------------------------------------------
# Kac / Clement
# --------------------------------------------------------------------------
def kac_clement(N: int = 10001, seed: int = 0) -> Problem:
    """Kac / Clement tridiagonal matrix of size N.

    Sub-diagonal A[i+1, i] = i + 1 and super-diagonal A[i, i+1] = N - 1 - i
    (i = 0..N-2), zero diagonal.  Its eigenvalues are -(N-1), -(N-3), ..., N-1,
    so it is singular for odd N.  x* ~ N(0,1), b = A x* (consistent).
    """
    i = np.arange(N - 1, dtype=np.int64)
    rows = np.concatenate([i + 1, i])
    cols = np.concatenate([i, i + 1])
    vals = np.concatenate([(i + 1).astype(np.float64), (N - 1 - i).astype(np.float64)])
    A = csr_from_coo(N, N, rows, cols, vals)
    xs = _rng("kac", seed).standard_normal(N)
    return Problem(f"kac_clement_{N}_s{seed}", A, A.matvec(xs), xs, {"N": N, "seed": seed})


# --------------------------------------------------------------------------
# LP-shaped wide matrix
# --------------------------------------------------------------------------
def lp_shaped(m: int = 10000, n: int = 1_000_000, per_col: int = 6, seed: int = 0,
              slack: bool = True) -> Problem:
    """A = S + [I_m 0]: S has ``per_col`` distinct uniformly drawn rows per
    column with N(0,1) values; the identity slack block sits on the first m
    columns (coinciding entries are summed).  x* ~ N(0,1), b = A x*."""
    if per_col > m:
        raise ValueError("per_col > m")
    g = _rng("lp", seed)
    rows = g.integers(0, m, size=(n, per_col))
    # Redraw repeated rows inside a column until all are distinct.
    while True:
        srt = np.sort(rows, axis=1)
        dup_cols = np.nonzero((srt[:, 1:] == srt[:, :-1]).any(axis=1))[0]
        if dup_cols.size == 0:
            break
        rows[dup_cols] = g.integers(0, m, size=(dup_cols.size, per_col))
    vals = g.standard_normal((n, per_col))
    cols = np.repeat(np.arange(n, dtype=np.int64), per_col)
    rr = rows.reshape(-1)
    vv = vals.reshape(-1)
    if slack:
        d = np.arange(min(m, n), dtype=np.int64)
        rr = np.concatenate([rr, d])
        cols = np.concatenate([cols, d])
        vv = np.concatenate([vv, np.ones(d.size)])
    A = csr_from_coo(m, n, rr, cols, vv)
    xs = g.standard_normal(n)
    return Problem(f"lp_shaped_{m}x{n}_s{seed}", A, A.matvec(xs), xs,
                   {"m": m, "n": n, "per_col": per_col, "seed": seed})


def skewed_rows(m: int, n: int, avg: float = 8.0, alpha: float = 1.5, seed: int = 0,
                empty_frac: float = 0.0, dense_rows: int = 0) -> Problem:
    """Row lengths Pareto(alpha) with mean ``avg`` (rounded, capped at n),
    a fraction ``empty_frac`` of the rows emptied, and ``dense_rows`` rows
    holding every column; columns uniform at random (repeats inside a row
    are summed), N(0,1) values.  x* ~ N(0,1), b = A x*."""
    g = _rng("skewed", seed)
    xm = avg * (alpha - 1.0) / alpha
    u = 1.0 - g.random(m)  # (0, 1]
    lens = np.minimum(np.rint(xm * u ** (-1.0 / alpha)), n).astype(np.int64)
    if empty_frac > 0.0:
        lens[g.random(m) < empty_frac] = 0
    if dense_rows > 0:
        lens[g.choice(m, size=min(dense_rows, m), replace=False)] = n
    rows = np.repeat(np.arange(m, dtype=np.int64), lens)
    cols = g.integers(0, n, size=rows.size)
    full = np.nonzero(lens == n)[0]
    if full.size:  # dense rows hold every column once
        starts = np.concatenate([[0], np.cumsum(lens)])[full]
        for s0 in starts:
            cols[s0:s0 + n] = np.arange(n)
    vals = g.standard_normal(rows.size)
    A = csr_from_coo(m, n, rows, cols, vals)
    xs = g.standard_normal(n)
    return Problem(f"skewed_{m}x{n}_s{seed}", A, A.matvec(xs), xs,
                   {"m": m, "n": n, "avg": avg, "alpha": alpha, "seed": seed,
                    "empty_frac": empty_frac, "dense_rows": dense_rows})


# --------------------------------------------------------------------------
# random diagonally dominant sparse
# --------------------------------------------------------------------------
def random_diag_dominant(n: int, offdiag: int = 7, seed: int = 0,
                         g: Optional[np.random.Generator] = None) -> Csr:
    """``offdiag`` distinct off-diagonal columns per row with N(0,1) values and
    a diagonal of 2 * sum |a_ij| over the row (nonsingular)."""
    g = _rng("randsparse", seed) if g is None else g
    k = min(offdiag, n - 1)
    cols = g.integers(0, n - 1, size=(n, k))
    while True:
        srt = np.sort(cols, axis=1)
        bad = np.nonzero((srt[:, 1:] == srt[:, :-1]).any(axis=1))[0] if k > 1 else np.array([], int)
        if bad.size == 0:
            break
        cols[bad] = g.integers(0, n - 1, size=(bad.size, k))
    r = np.arange(n, dtype=np.int64)[:, None]
    cols = cols + (cols >= r)  # skip the diagonal
    vals = g.standard_normal((n, k))
    diag = 2.0 * np.abs(vals).sum(axis=1)
    rows = np.concatenate([np.repeat(np.arange(n), k), np.arange(n)])
    cc = np.concatenate([cols.reshape(-1), np.arange(n)])
    vv = np.concatenate([vals.reshape(-1), diag])
    return csr_from_coo(n, n, rows, cc, vv)


# --------------------------------------------------------------------------
# batched uneven systems
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Batch:
    systems: List[Csr]
    B: List[np.ndarray]  # column-major n_s x k_s blocks, as (n_s, k_s) float64 arrays
    kinds: List[str]
    meta: dict


def batched_uneven(nsys: int = 256, nmin: int = 1024, nmax: int = 65536, kmin: int = 1,
                   kmax: int = 64, seed: int = 0) -> Batch:
    """Uneven batch: half Poisson 5-point stencils (nx = floor(sqrt(n)),
    ny = ceil(n / nx)), half random sparse with 7 off-diagonals plus a dominant
    diagonal.  Each system gets k ~ U{kmin..kmax} right-hand sides ~ U[-1, 1]."""
    g = _rng("batched", seed)
    systems, Bs, kinds = [], [], []
    for s in range(nsys):
        n = int(g.integers(nmin, nmax + 1))
        k = int(g.integers(kmin, kmax + 1))
        if s % 2 == 0:
            nx = int(math.isqrt(n))
            ny = -(-n // nx)
            A = poisson5(nx, ny)
            kinds.append("stencil")
        else:
            A = random_diag_dominant(n, 7, g=g)
            kinds.append("random")
        systems.append(A)
        Bs.append(g.uniform(-1.0, 1.0, (A.m, k)))
    return Batch(systems, Bs, kinds, {"nsys": nsys, "seed": seed})


def ladder():
    """Small inputs on which the oracle finishes in seconds."""
    return [
        dense_gaussian(20, seed=0),
        dense_gaussian(50, seed=1),
        convection_diffusion(8),
        convection_diffusion(16),
        kac_clement(101),
        kac_clement(1001),
        lp_shaped(200, 5000, seed=0),
    ]
