"""Backward pass: gradients of Re<eta, g(H_W) b> for the links and mu,
against the oracle's dense reference gradient, finite differences, and
through torch.autograd."""
import json
import os

import numpy as np
import pytest

import skinputs as si
from skinputs.configs import CONFIGS
from oracle import gradient, rational
from tests.gpu_util import make_op, to_dev, from_dev, rel, announce, torch_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 2, 3, 4)])
def test_gradient_matches_dense_oracle_every_coordinate(dims):
    from paper_0910_2927_amd import api
    V = si.lattice_volume(dims)
    U = si.gauge_links(dims, 0.5, 600 + V)
    b = si.gaussian_source(12 * V, 601)
    eta = si.gaussian_source(12 * V, 602)
    sig, om = rational.kl_first_order(5, 1.3)
    announce(f"backward dims={dims}")
    op = make_op(U, dims, 0.25, 0.3)
    x, g, gmu = api.sign_apply_backward(op, to_dev(b, V), to_dev(eta, V), sig, om, 16, tol=1e-13)
    ref, refmu = gradient.dense_gradient(U, dims, 0.25, 0.3, b, eta, sig, om)
    G = g.cpu().numpy()
    R = np.zeros_like(G)
    for (nu, s, a), v in ref.items():
        R[nu, s, a] = v
    assert np.abs(G - R).max() <= 1e-9 * np.abs(R).max()
    assert abs(gmu - refmu) <= 1e-8 * max(1.0, abs(refmu))


def test_gradient_4x4_directional_and_sampled_coordinates():
    from paper_0910_2927_amd import api
    dims = (4, 4, 4, 4)
    V = 256
    U = si.gauge_links(dims, 0.5, 610)
    b = si.gaussian_source(12 * V, 611)
    eta = si.gaussian_source(12 * V, 612)
    sig, om = rational.kl_first_order(8, 1.4)
    announce("backward 4^4")
    op = make_op(U, dims, 0.25, 0.3)
    _, g, gmu = api.sign_apply_backward(op, to_dev(b, V), to_dev(eta, V), sig, om, 30, tol=1e-13)
    G = g.cpu().numpy()
    theta = si.su3_directions(V, si.seed_for(4, "dir"))
    dd = gradient.directional_dense(U, dims, 0.25, 0.3, b, eta, sig, om, theta)
    assert abs(np.sum(G * theta) - dd) <= 1e-9 * abs(dd)
    coords = [(0, 5, 3), (3, 200, 7), (2, 255, 0)]
    ref, refmu = gradient.dense_gradient(U, dims, 0.25, 0.3, b, eta, sig, om, coords=coords)
    for c in coords:
        assert abs(G[c] - ref[c]) <= 1e-9 * np.abs(G).max()
    assert abs(gmu - refmu) <= 1e-8 * max(1.0, abs(refmu))


def test_config_cg_8x4_central_differences_and_autograd():
    """8^4, mu = 0.3, 16 poles, k = 50: the directional derivative along a
    random su(3) direction and d/dmu against central differences (h = 1e-5)
    of F evaluated by the library's forward solves; the forward result
    against the oracle's stored x*; the same gradient via torch.autograd."""
    import torch
    from paper_0910_2927_amd import api
    cfg = CONFIGS["cg"]
    mu = 0.3
    c = cfg.scales[mu]
    g = json.load(open(os.path.join(GOLDEN, f"cg_mu{mu:g}.json")))
    U = si.gauge_links(cfg.dims, cfg.eps, si.seed_for(cfg.L, "gauge"))
    b = si.gaussian_source(cfg.n, si.seed_for(cfg.L, "b"))
    eta = si.gaussian_source(cfg.n, si.seed_for(cfg.L, "eta"))
    sig, om = api.kl_poles(cfg.s, c)
    op = make_op(U, cfg.dims, cfg.kappa, mu)
    bd, ed = to_dev(b, cfg.V), to_dev(eta, cfg.V)
    announce("backward cg 8^4")
    x, G, gmu = api.sign_apply_backward(op, bd, ed, sig, om, cfg.k, tol=1e-14, max_cycles=2000)
    idx = np.array(g["sample_index"])
    xh = from_dev(x, cfg.V)
    assert rel(xh[idx], np.array(g["x_re"]) + 1j * np.array(g["x_im"])) <= 1e-8
    full = os.path.join(GOLDEN, f"cg_mu{mu:g}_x.npy")
    if os.path.exists(full):
        assert rel(xh, np.load(full)) <= 1e-8
    theta = si.su3_directions(cfg.V, si.seed_for(cfg.L, "dir"))
    h = 1e-5

    def F(Ul, mul):
        o = make_op(Ul, cfg.dims, cfg.kappa, mul)
        r = api.sign_apply(o, bd, sig, om, cfg.k, tol=1e-14, max_cycles=2000)
        return float(np.real(np.vdot(eta, from_dev(r.x, cfg.V))))

    announce("backward cg 8^4: finite differences")
    fd = (F(gradient.rotate_links(U, theta, h), mu) - F(gradient.rotate_links(U, theta, -h), mu)) / (2 * h)
    an = float((G.cpu().numpy() * theta).sum())
    print(f"directional: analytic {an:.12e} central FD {fd:.12e} rel {abs(an - fd) / abs(fd):.2e}")
    assert abs(an - fd) <= 1e-6 * abs(fd)
    fdmu = (F(U, mu + h) - F(U, mu - h)) / (2 * h)
    print(f"mu: analytic {gmu:.12e} central FD {fdmu:.12e}")
    assert abs(gmu - fdmu) <= 1e-6 * max(1.0, abs(fdmu))
    # torch.autograd route: loss = Re <eta, x>
    theta_t = torch.zeros((4, cfg.V, 8), dtype=torch.float64, device=torch_dev(), requires_grad=True)
    mu_t = torch.tensor(mu, dtype=torch.float64, device=torch_dev(), requires_grad=True)
    xo = api.SignKrylov.apply(theta_t, mu_t, bd, op, sig, om, cfg.k, 1e-14, 2000)
    loss = (torch.conj(ed) * xo).sum().real
    loss.backward()
    assert torch.allclose(theta_t.grad, G, rtol=0, atol=1e-10 * float(G.abs().max()))
    assert abs(float(mu_t.grad) - gmu) <= 1e-10 * max(1.0, abs(gmu))
