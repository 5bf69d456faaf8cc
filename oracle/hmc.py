"""Plain FP64 oracle of a hybrid-Monte-Carlo molecular-dynamics trajectory.

TEST INFRASTRUCTURE ONLY: used by tests/ to check the HIP path; the product
library never imports it.  Shares no code with the HIP path.

What it follows.  The paper (Sec. 4) reports hybrid Monte Carlo gauge
generation with the staggered operator as nearly complete and prints no
formula; the definitions are the textbook ones:

  Wilson gauge action  S_g(U) = beta sum_x sum_{mu<nu} [1 - Re tr P_munu(x) / 3],
                       P_munu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
  pseudofermion action S_f(U) = phi^dag A(U)^-1 phi  (one even-site field)
  momenta              p^a_mu(x), a = 1..8, P = sum_a p^a T_a, T_a = lambda_a / 2
  Hamiltonian          H = 1/2 sum p^2 + S_g + S_f
  flow                 U <- exp(i eps P) U,   p^a <- p^a - eps F^a,
                       F^a = d/dw S(exp(i w T_a) U) at w = 0
  leapfrog             p half step; (U step, p step) n - 1 times; U step; p half step

Link gradients follow the library's convention G = dS/dRe U + i dS/dIm U, so
F^a = Re[i tr(T_a U G^dag)] (oracle.su3_force).  For the gauge action
G_mu(x) = -(beta/3) A_mu(x)^dag with A_mu(x) the sum of the six staples.

Layouts: U (4, V, 3, 3) complex128 lexicographic (x0 fastest), p (4, V, 8).
Parity status: pinned in tests/test_oracle_hmc.py (closed forms, gauge
invariance, finite differences, scipy's expm, reversibility, the order of the
integrator's energy error).
"""
from __future__ import annotations

import numpy as np

import oracle


def _grid(dims, a):
    """(V, ...) -> (L3, L2, L1, L0, ...): lexicographic order with x0 fastest."""
    L0, L1, L2, L3 = dims
    return a.reshape((L3, L2, L1, L0) + a.shape[1:])


def _shift(dims, a, mu, step):
    """b(x) = a(x + step * mu) on the grid form (periodic)."""
    return np.roll(a, -step, axis=3 - mu)


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def gauge_action(dims, U, beta):
    """S_g = beta sum_{x, mu<nu} (1 - Re tr P_munu(x) / 3)."""
    Ug = [_grid(dims, U[mu]) for mu in range(4)]
    s = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            P = Ug[mu] @ _shift(dims, Ug[nu], mu, 1) @ _dag(_shift(dims, Ug[mu], nu, 1)) @ _dag(Ug[nu])
            s += np.sum(1.0 - np.real(np.trace(P, axis1=-2, axis2=-1)) / 3.0)
    return beta * s


def staples(dims, U):
    """A_mu(x) = sum_{nu != mu} [U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
                                 + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)], (4, V, 3, 3)."""
    Ug = [_grid(dims, U[mu]) for mu in range(4)]
    out = np.zeros_like(U)
    for mu in range(4):
        A = np.zeros_like(Ug[mu])
        for nu in range(4):
            if nu == mu:
                continue
            up = _shift(dims, Ug[nu], mu, 1) @ _dag(_shift(dims, Ug[mu], nu, 1)) @ _dag(Ug[nu])
            lo_nu = _shift(dims, Ug[nu], nu, -1)                      # U_nu(x - nu)
            lo = _dag(_shift(dims, lo_nu, mu, 1)) @ _dag(_shift(dims, Ug[mu], nu, -1)) @ lo_nu
            A += up + lo
        out[mu] = A.reshape(U[mu].shape)
    return out


def gauge_grad(dims, U, beta):
    """G = dS_g/dRe U + i dS_g/dIm U = -(beta/3) A^dag."""
    return -(beta / 3.0) * _dag(staples(dims, U))


def su3_exp(eps, p):
    """exp(i eps P), P = sum_a p^a T_a (Hermitian, traceless), by the eigen-decomposition."""
    T = oracle.gell_mann() / 2.0
    P = np.einsum("...a,aij->...ij", p, T)
    w, v = np.linalg.eigh(P)
    return (v * np.exp(1j * eps * w)[..., None, :]) @ _dag(v)


def link_update(U, p, eps):
    return su3_exp(eps, p) @ U


def kinetic(p):
    return 0.5 * float(np.sum(p * p))


def total_force(dims, U, beta, phi, mass, tol=1e-13):
    """(F^a of S_g + S_f (4, V, 8), S_f)."""
    G = gauge_grad(dims, U, beta)
    S_f = 0.0
    if phi is not None:
        S_f, Gf, _, _ = oracle.force(dims, U, mass, phi, tol=tol)
        G = G + Gf
    return oracle.su3_force(U, G), S_f


def md_trajectory(dims, U, p, phi, beta, mass, eps, nsteps, tol=1e-13):
    """Leapfrog trajectory; returns (U, p, H_start, H_end, per-force S_f list)."""
    U = U.copy()
    p = p.copy()
    F, S_f0 = total_force(dims, U, beta, phi, mass, tol)
    H0 = kinetic(p) + gauge_action(dims, U, beta) + S_f0
    p = p - 0.5 * eps * F
    S_f = S_f0
    for i in range(nsteps):
        U = link_update(U, p, eps)
        F, S_f = total_force(dims, U, beta, phi, mass, tol)
        p = p - (eps if i < nsteps - 1 else 0.5 * eps) * F
    H1 = kinetic(p) + gauge_action(dims, U, beta) + S_f
    return U, p, H0, H1
