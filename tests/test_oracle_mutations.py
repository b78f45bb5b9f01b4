"""Planted mistakes in the oracle must fail at least one pin.

Each case swaps one oracle function for a plausibly wrong variant (a dropped
term, a wrong sign, a transposed operand, a wrong index) and runs the pins
that should catch it.  Everything here runs on the CPU.
"""
import numpy as np
import pytest

from oracle import certificate, embedding, jl_signs, pca
import tests.test_oracle_pins as pins


def _fails(fn):
    try:
        fn()
    except AssertionError:
        return True
    return False


def _wrong_sign_sq(Vt, r, seed):
    d = Vt.shape[1]
    s, k = embedding.split(r, d)
    P = Vt[:s]
    if k == 0:
        return P.copy()
    S = jl_signs.jl_matrix(seed, k, d)
    return np.vstack([P, S + (S @ P.T) @ P])


def _transposed_tp(Vt, r, seed):
    d = Vt.shape[1]
    s, k = embedding.split(r, d)
    P = Vt[:s]
    if k == 0:
        return P.copy()
    S = jl_signs.jl_matrix(seed, k, d)
    return np.vstack([P, S - S @ (P.T @ P).T @ P.T @ P])  # projects twice: harmless


def _ascending_axes(C):
    lam, V = np.linalg.eigh(C)
    return lam, V.T.copy()


def _uncentred_pca(X):
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=0)
    C = X.T @ X
    lam, Vt = pca.principal_axes(C)
    return mu, C, lam, Vt


_certify = certificate.certify


def _squared_ratio_certify(X, Y, rows=None):
    c = _certify(X, Y, rows)
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    I, J = c["i"], c["j"]
    if I >= 0:
        D2 = np.sum((X[I] - X[J]) ** 2)
        E2 = np.sum((Y[I] - Y[J]) ** 2)
        c["max"] = abs(E2 / D2 - 1)
    return c


def _scaled_signs(seed, k, d):
    return jl_signs.sign_matrix(seed, k, d) / k


def _swapped_split(r, d):
    if r == d:
        return d, 0
    return r - r // 2, r // 2


def _bit0_signs(seed, k, d):
    a = np.arange(k, dtype=np.uint64)[:, None]
    l = np.arange(d, dtype=np.uint64)[None, :]
    z = jl_signs.splitmix64_output(seed, ((a << np.uint64(32)) | l) + np.uint64(1))
    return np.where((z & np.uint64(1)) == 0, 1.0, -1.0)


def test_wrong_sign_in_sq_is_caught(monkeypatch):
    monkeypatch.setattr(embedding, "adagio_map", _wrong_sign_sq)
    assert _fails(pins.test_exact_rank_data_has_zero_distortion)
    assert _fails(pins.test_map_structure)


def test_harmless_reassociation_passes(monkeypatch):
    """Control: an algebraically identical SQ must still pass."""
    monkeypatch.setattr(embedding, "adagio_map", _transposed_tp)
    pins.test_map_structure()
    pins.test_exact_rank_data_has_zero_distortion()


def test_ascending_eigen_order_is_caught(monkeypatch):
    monkeypatch.setattr(pca, "principal_axes", _ascending_axes)
    assert _fails(pins.test_principal_axes_residual_and_order)
    assert _fails(pins.test_pca_minimises_eq4)
    assert _fails(pins.test_pca_only_distortion_bound)


def test_missing_centring_is_caught(monkeypatch):
    monkeypatch.setattr(pca, "pca", _uncentred_pca)
    assert _fails(pins.test_covariance_equals_pairwise_secant_sum)


def test_squared_distortion_is_caught(monkeypatch):
    monkeypatch.setattr(certificate, "certify", _squared_ratio_certify)
    assert _fails(pins.test_certificate_two_points_closed_form)


def test_wrong_jl_scale_is_caught(monkeypatch):
    monkeypatch.setattr(jl_signs, "jl_matrix", _scaled_signs)
    assert _fails(pins.test_jl_moments_rademacher)
    assert _fails(pins.test_map_structure)


def test_swapped_split_is_caught(monkeypatch):
    monkeypatch.setattr(embedding, "split", _swapped_split)
    assert _fails(pins.test_split_rule)


def test_wrong_sign_bit_is_caught(monkeypatch):
    monkeypatch.setattr(jl_signs, "sign_matrix", _bit0_signs)
    assert _fails(pins.test_sign_matrix_counter_layout)
