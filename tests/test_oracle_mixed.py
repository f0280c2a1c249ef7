"""Pins of the oracle's mixed-precision helpers (scaled cast, LANSF norms)
against closed forms and library routines."""
import numpy as np
import pytest

import oracle
import synth

LAYOUTS = oracle.LAYOUTS


def _unit_diag_spd(n, seed):
    """C with an exactly unit diagonal: a correlation-like SPD matrix."""
    A, _ = synth.spd(n, seed=seed)
    d = np.sqrt(np.diag(A))
    C = A / d[:, None] / d[None, :]
    C = 0.5 * (C + C.T)
    C[np.diag_indices(n)] = 1.0
    return np.asfortranarray(C)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [1, 2, 7, 64, 129])
def test_cast_without_scaling_is_plain_rounding(transr, uplo, n):
    """scale off, mu = 1: the cast is numpy's binary64 -> binary32 rounding."""
    A, _ = synth.spd(n, seed=n)
    arf = oracle.trttf(transr, uplo, A)
    s, out = oracle.pfcast_s(transr, uplo, n, arf, scale=False, mu=1.0)
    assert np.array_equal(s, np.ones(n))
    assert np.array_equal(out, arf.astype(np.float32))


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [2, 7, 64, 129])
@pytest.mark.parametrize("mu", [1.0, 4096.0])
def test_cast_undoes_power_of_two_scaling_exactly(transr, uplo, n, mu):
    """A = D0 C D0 with D0 = diag(2^e) and unit-diagonal C: diag(A) = 4^e, so
    s = 2^-e exactly and the scaled matrix is mu C with no rounding in FP64."""
    C = _unit_diag_spd(n, seed=n + 1)
    e = synth.rng(n).integers(-20, 21, size=n)
    d0 = np.ldexp(1.0, e)
    A = np.asfortranarray(d0[:, None] * C * d0[None, :])
    arf = oracle.trttf(transr, uplo, A)
    s, out = oracle.pfcast_s(transr, uplo, n, arf, scale=True, mu=mu)
    assert np.array_equal(s, np.ldexp(1.0, -e))
    want = oracle.trttf(transr, uplo, np.asfortranarray(C * mu)).astype(np.float32)
    assert np.array_equal(out, want)


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [1, 7, 129])
@pytest.mark.parametrize("shift", [2.0 ** -9, 2.0 ** -6])
def test_cast_shift_adds_to_the_unit_diagonal(transr, uplo, n, shift):
    """Same exact setting as above: the scaled matrix is mu (C + shift I),
    and with shift and mu powers of two and C's diagonal 1 every stored
    value is still exact (1 + shift fits in FP32's 24 bits)."""
    C = _unit_diag_spd(n, seed=n + 3)
    e = synth.rng(n + 5).integers(-10, 11, size=n)
    d0 = np.ldexp(1.0, e)
    A = np.asfortranarray(d0[:, None] * C * d0[None, :])
    mu = 4096.0
    arf = oracle.trttf(transr, uplo, A)
    s, out = oracle.pfcast_s(transr, uplo, n, arf, scale=True, mu=mu, shift=shift)
    want = oracle.trttf(transr, uplo, np.asfortranarray(mu * (C + shift * np.eye(n)))).astype(np.float32)
    assert np.array_equal(out, want)
    # the off-diagonal entries are those of the unshifted cast
    _, out0 = oracle.pfcast_s(transr, uplo, n, arf, scale=True, mu=mu)
    diag = oracle.trttf(transr, uplo, np.asfortranarray(np.eye(n))) != 0
    assert np.array_equal(out[~diag], out0[~diag])
    assert np.all(out[diag] == np.float32(mu * (1.0 + shift)))


def test_cast_marks_non_positive_diagonal():
    n = 9
    A, _ = synth.spd(n, seed=2)
    A[4, 4] = -1.0
    A[6, 6] = 0.0
    s, out = oracle.pfcast_s("N", "L", n, oracle.trttf("N", "L", A), scale=True)
    assert np.isnan(s[4]) and np.isnan(s[6])
    assert np.all(np.isfinite(np.delete(s, [4, 6])))


@pytest.mark.parametrize("transr,uplo", LAYOUTS)
@pytest.mark.parametrize("n", [1, 2, 7, 50, 65])
def test_norms_against_numpy(transr, uplo, n):
    A, _ = synth.spd(n, seed=n + 9)
    A[0, -1] = A[-1, 0] = -3.5  # a negative entry
    arf = oracle.trttf(transr, uplo, A)
    assert oracle.norm_max(transr, uplo, n, arf) == np.abs(A).max()
    assert abs(oracle.norm_fro(transr, uplo, n, arf) - np.linalg.norm(A)) <= 1e-14 * np.linalg.norm(A)
    assert abs(oracle.norm_inf(transr, uplo, n, arf) - np.linalg.norm(A, np.inf)) <= 1e-14 * np.linalg.norm(A, np.inf)
