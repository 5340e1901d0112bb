"""Helpers shared by the GPU parity tests (no sampler arithmetic here)."""
import numpy as np
import pytest

import synth


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1608_04329_amd import hsp
    hsp.load()
    return torch, hsp


def dataset(N, p, seed, k_nonzero=None):
    """Probit design with an intercept; a few nonzero coefficients."""
    if k_nonzero is None:
        k_nonzero = min(5, p - 1)
    beta, _ = synth.sparse_beta(p, k_nonzero, seed, -2.0, 2.0)
    return synth.probit_design(N, p, beta, seed, True, f"n{N}_p{p}")


def random_state(p, seed, beta_scale=0.3):
    rng = np.random.default_rng(seed)
    return dict(beta=rng.normal(0, beta_scale, p), lam_m2=rng.gamma(2.0, 1.0, p),
                nu_m1=rng.gamma(2.0, 1.0, p), tau_m2=float(rng.gamma(3.0, 1.0)),
                xi_m1=float(rng.gamma(2.0, 1.0)))


def z_scale(X, beta):
    """Natural scale of each latent draw: max(sum_j |x_ij beta_j|, 1)."""
    return np.maximum(np.abs(X.astype(np.float64)) @ np.abs(beta), 1.0)


def b_scale(X, z):
    """Condition scale of X^T z: sum_i |x_ij z_i|."""
    return np.abs(X.astype(np.float64)).T @ np.abs(z)
