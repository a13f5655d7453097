"""Oracle: the Kenney-Laub / Neuberger rational approximation of sign.

TEST INFRASTRUCTURE ONLY.

Sect. 6 approximates sign(t) by
    g_s(t) = ((t+1)^{2s} - (t-1)^{2s}) / ((t+1)^{2s} + (t-1)^{2s})
and quotes its partial-fraction expansion in t^2,
    g_s(t) = t * sum_{i=1..s} w_i / (t^2 - q_i),
    w_i = 1/(s cos^2(theta_i)),  q_i = -tan^2(theta_i),  theta_i = pi (i - 1/2) / (2 s),
used as g_s(c t) with a scale c > 0 (two-circle formula c = ((m+r)(m-r))^{-1/2}).

Eq. (g) of Sect. 2 and Algorithm 1 work with first-order poles,
g(x) = sum_j omega_j / (x - sigma_j).  Splitting
t/(t^2 + tau^2) = 1/2 [1/(t - i tau) + 1/(t + i tau)] turns g_s(c x) into
N = 2s first-order terms with
    sigma = +- i tau_i / c,   omega = w_i / (2 c),   tau_i = tan(theta_i).
The pole set is closed under complex conjugation and all weights are real.
"""
from __future__ import annotations

import numpy as np

__all__ = ["kl_closed_form", "kl_t2_terms", "kl_t2_form", "kl_first_order",
           "g_first_order"]


def kl_closed_form(t, s: int):
    """g_s(t) as the ratio of (t+1)^{2s} -+ (t-1)^{2s} (Sect. 6).

    Evaluated as (1 - z)/(1 + z) with z = ((t-1)/(t+1))^{2s}, which is the
    same rational function divided through by (t+1)^{2s}."""
    t = np.asarray(t, dtype=np.complex128)
    z = ((t - 1) / (t + 1)) ** (2 * s)
    return (1 - z) / (1 + z)


def kl_t2_terms(s: int):
    """(w_i, q_i), i = 1..s, of the t^2 partial fractions (Sect. 6)."""
    i = np.arange(1, s + 1)
    th = np.pi / (2 * s) * (i - 0.5)
    w = 1.0 / (s * np.cos(th) ** 2)
    q = -np.tan(th) ** 2
    return w, q


def kl_t2_form(t, s: int):
    t = np.asarray(t, dtype=np.complex128)
    w, q = kl_t2_terms(s)
    return t * sum(wi / (t * t - qi) for wi, qi in zip(w, q))


def kl_first_order(s: int, c: float = 1.0):
    """First-order poles and weights of g_s(c x): arrays sigma[2s], omega[2s].

    Order: for i = 1..s the pair (+i tau_i / c, -i tau_i / c)."""
    w, q = kl_t2_terms(s)
    tau = np.sqrt(-q)
    sigma = np.empty(2 * s, dtype=np.complex128)
    omega = np.empty(2 * s, dtype=np.complex128)
    sigma[0::2] = 1j * tau / c
    sigma[1::2] = -1j * tau / c
    omega[0::2] = w / (2 * c)
    omega[1::2] = w / (2 * c)
    return sigma, omega


def g_first_order(x, sigma, omega):
    """Eq. (g): g(x) = sum_j omega_j / (x - sigma_j)."""
    x = np.asarray(x, dtype=np.complex128)
    return sum(o / (x - s_) for s_, o in zip(sigma, omega))

