"""Pins of the oracle's transposed pFFT operator and of its sigma gradient.

* Transpose: y^T (A~ x) = x^T (A~^T y) for random x, y (the forward operator
  is pinned elsewhere, so this fixes the transpose).
* Gradient: the adjoint formula d f/d c_k = 2 Re[lam^T (db/dc_k - dA/dc_k x)],
  A^T lam = g, for the reflected-amplitude objective of the differentiation
  workload, against central finite differences of the objective computed by
  full re-solves -- for the dense Galerkin matrix and for the pFFT operator.
"""
import copy

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


@pytest.fixture(scope="module")
def setup():
    w = synth.workload_gradient(guide_len=0.8, absorber=1.2, edge=0.15, n_ctrl=8, n_monitor=6)
    o = oracle.Oracle(w.mesh, w.omega, w.eps_in)
    o.set_sigma(w.sigma)
    d = w.dipoles[0]
    xs = w.notes["monitor_x"]
    pts = np.stack([xs, np.zeros_like(xs), np.zeros_like(xs)], 1)
    wts = oracle.monitor_weights(xs, w.notes["beta"])
    Einc = np.array([oracle.dipole_field(o.k_i, o.Z_i, d.pos, d.moment, p)[0] for p in pts])
    Q = o.field_matrix(pts, 0).reshape(len(xs), 3, o.N)[:, 1, :]
    return w, o, wts @ Q, wts @ Einc[:, 1]


def test_monitor_weights_recover_amplitudes():
    xs = np.linspace(0.3, 2.9, 9)
    beta = 4.1
    E = (0.7 - 0.2j) * np.exp(-1j * beta * xs) + (-0.3 + 0.45j) * np.exp(1j * beta * xs)
    assert abs(oracle.monitor_weights(xs, beta) @ E - (-0.3 + 0.45j)) < 1e-12


def test_pfft_transpose_bilinear(setup):
    w, o, _, _ = setup
    P = o.pfft(w.h, w.r_near)
    rng = np.random.default_rng(5)
    for _ in range(2):
        x = rng.standard_normal(o.N) + 1j * rng.standard_normal(o.N)
        y = rng.standard_normal(o.N) + 1j * rng.standard_normal(o.N)
        a, b = y @ P.matvec(x), x @ P.rmatvec(y)
        assert abs(a - b) <= 1e-12 * abs(a)


def _objective(w, o, q, c0, ctrl, mode):
    e2 = copy.copy(w.sigma[0])
    e2.ctrl = ctrl
    o.set_sigma([e2])
    b = o.rhs_dipole(w.dipoles[0])
    if mode == "dense":
        x = oracle.lu_solve(o.dense(), b)
    else:
        x = o.pfft(w.h, w.r_near).solve(b, tol=1e-13)
    bh = c0 + q @ x
    return abs(bh) ** 2, bh, x


@pytest.mark.parametrize("mode", ["dense", "pfft"])
def test_gradient_matches_central_differences(setup, mode):
    w, o, q, c0 = setup
    end = w.sigma[0]
    f0, bh, x = _objective(w, o, q, c0, end.ctrl, mode)
    g = np.conj(bh) * q                      # d f / d x with df = 2 Re(g^T dx)
    Einc, _ = o.incident_at_points(w.dipoles[0])
    if mode == "dense":
        lam = oracle.lu_solve(o.dense().T, g)
        Ee, Ei = o.point_fields(x)
    else:
        P = o.pfft(w.h, w.r_near)
        lam = P.solve_t(g, tol=1e-13)
        Ee, Ei = P.point_fields(x)
    grad = o.pwl_jacobian(end).T @ o.sigma_gradient_points(lam, Ee, Ei, Einc)
    scale = np.max(np.abs(grad))
    dl = 1e-5
    for k in (0, 3):
        cp, cm = end.ctrl.copy(), end.ctrl.copy()
        cp[k] += dl
        cm[k] -= dl
        fd = (_objective(w, o, q, c0, cp, mode)[0] - _objective(w, o, q, c0, cm, mode)[0]) / (2 * dl)
        assert abs(fd - grad[k]) <= 2e-6 * scale, (k, fd, grad[k])
    # a dropped incident-field term (db/dsigma) is visible at this size
    wrong = o.pwl_jacobian(end).T @ o.sigma_gradient_points(lam, Ee, Ei, None)
    assert np.max(np.abs(wrong - grad)) > 1e-3 * scale
    o.set_sigma(w.sigma)
