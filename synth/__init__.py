"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws numbers and builds dense symmetric positive definite
matrices in ordinary full (column-major) storage.  It holds none of the RFP
method's arithmetic: packing into RFP, factoring and solving happen on each
side with that side's own code.

Recipe (the paper never states how its SPD test matrices were made):
    rng = numpy.random.Generator(PCG64(seed))
    M   = rng.standard_normal((n, k))        # drawn first
    B   = rng.standard_normal((n, nrhs))     # drawn second
    A   = M M^T / k, symmetrised as (A + A^T)/2, plus alpha on the diagonal.
For n >= 8192 the product M M^T may be formed on the GPU by torch (input
synthesis only; not part of the measured path).
"""
import math

import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def spd(n, k=None, alpha=1.0, nrhs=0, seed=0):
    """A = M M^T / k + alpha I (n x n, Fortran order) and B (n x nrhs)."""
    k = n if k is None else k
    g = rng(seed)
    M = g.standard_normal((n, k))
    B = np.asfortranarray(g.standard_normal((n, nrhs))) if nrhs else None
    A = M @ M.T
    A /= k
    A = 0.5 * (A + A.T)
    A[np.diag_indices(n)] += alpha
    return np.asfortranarray(A), B


def spd_device(n, k=None, alpha=1.0, nrhs=0, seed=0, device="cuda"):
    """Same recipe as :func:`spd`, with the n x n product formed by torch on
    ``device``.  Returns torch tensors: A (column-major, shape (n, n) with
    strides (1, n)) and B (shape (n, nrhs), column-major), both float64."""
    import torch

    k = n if k is None else k
    g = rng(seed)
    M = torch.from_numpy(g.standard_normal((n, k))).to(device)
    B = None
    if nrhs:
        B = torch.from_numpy(np.asfortranarray(g.standard_normal((n, nrhs)))).to(device)
        B = B.t().contiguous().t()
    A = M @ M.t()
    del M
    A.div_(k)
    A = 0.5 * (A + A.t())
    A.diagonal().add_(alpha)
    A = A.t().contiguous().t()  # column-major (symmetric anyway)
    return A, B


def hpd(n, k=None, alpha=1.0, nrhs=0, seed=0):
    """Complex Hermitian A = M M^H / k + alpha I, M with N(0,1) real and
    imaginary parts (n x n complex128, Fortran order, real diagonal), and
    complex B (n x nrhs)."""
    k = n if k is None else k
    g = rng(seed)
    M = g.standard_normal((n, k)) + 1j * g.standard_normal((n, k))
    B = None
    if nrhs:
        B = np.asfortranarray(g.standard_normal((n, nrhs)) + 1j * g.standard_normal((n, nrhs)))
    A = M @ M.conj().T
    A /= k
    A = 0.5 * (A + A.conj().T)
    A[np.diag_indices(n)] = A[np.diag_indices(n)].real + alpha
    return np.asfortranarray(A), B


def hpd_device(n, k=None, alpha=1.0, nrhs=0, seed=0, device="cuda"):
    """Same recipe as :func:`hpd` with the product formed by torch on
    ``device``; complex128 tensors, column-major."""
    import torch

    k = n if k is None else k
    g = rng(seed)
    M = torch.from_numpy(g.standard_normal((n, k)) + 1j * g.standard_normal((n, k))).to(device)
    B = None
    if nrhs:
        B = torch.from_numpy(np.asfortranarray(g.standard_normal((n, nrhs)) + 1j * g.standard_normal((n, nrhs))))
        B = B.to(device).t().contiguous().t()
    Mh = M.conj().t().contiguous()
    A = M @ Mh
    del M, Mh
    A.div_(k)
    A = 0.5 * (A + A.conj().t())
    A.diagonal().copy_(A.diagonal().real + alpha)
    A = A.t().contiguous().t()
    return A, B


def rhs(n, nrhs, seed):
    """Standalone right-hand sides N(0,1), column-major."""
    return np.asfortranarray(rng(seed).standard_normal((n, nrhs)))


def min_matrix(n, dtype=np.float64):
    """a_ij = min(i, j) + 1 (0-based).  Its Cholesky factor is the all-ones
    lower triangle, its inverse is tridiag(-1, 2, -1) with a last diagonal
    entry of 1; every intermediate value is a small integer."""
    i = np.arange(n)
    return np.asfortranarray(np.minimum.outer(i, i).astype(dtype) + 1)


def scaled_min_matrix(n, seed=0, emax=6):
    """D A D with A the min matrix and D = diag(2^e_i), e_i in [-emax, emax].
    Its factor is D times the all-ones lower triangle, exactly."""
    e = rng(seed).integers(-emax, emax + 1, size=n)
    d = np.ldexp(1.0, e)
    return np.asfortranarray(d[:, None] * min_matrix(n) * d[None, :]), d


def cond_alpha(n, k, kappa):
    """alpha giving cond(M M^T/k + alpha I) ~ kappa for n > k (rank-deficient
    Gram part, smallest eigenvalue alpha): the largest eigenvalue of M M^T/k is
    taken at its Marchenko-Pastur edge (1 + sqrt(n/k))^2."""
    lmax = (1.0 + math.sqrt(n / k)) ** 2
    return lmax / (kappa - 1.0)


def batch_sizes(count, nmin, nmax, rmin, rmax, seed, log_uniform=False):
    """Sizes, layouts and right-hand-side counts for a batch of systems.
    Draw order: all n_i, then all layouts, then all nrhs_i."""
    g = rng(seed)
    if log_uniform:
        ns = np.rint(np.exp(g.uniform(math.log(nmin), math.log(nmax), size=count))).astype(np.int64)
    else:
        ns = g.integers(nmin, nmax + 1, size=count)
    lay = g.integers(0, 4, size=count)
    nr = g.integers(rmin, rmax + 1, size=count)
    return ns, lay, nr
