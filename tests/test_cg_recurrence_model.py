"""A NumPy model of two CG recurrences with FP32 inner iterations and FP64
reliable updates, as the solver runs them (independent CG per source, the
update trigger |r| < delta max|r|, p kept across an update with
beta = |r_new|^2 / |r_old|^2).  It backs a design decision, not the library:
the recurrence of the engines (classical CG, Sec. 4's CG benchmark) against
the pipelined single-reduction recurrence of Ghysels and Vanroose (2014),
whose matrix-vector product does not wait for the step's sums (w = A r,
s = A p and z = A s kept by recurrences, one fused reduction of |r|^2 and
<w, r> per step).  In FP32 the pipelined recurrence needs more iterations on a
matrix with the spectrum of a light-mass Dirac normal operator, which cancels
the latency it would hide; in FP64 it needs no more.  No GPU and no oracle."""
import numpy as np
import pytest

N = 400
TOL, DELTA = 1e-10, 0.1


@pytest.fixture(scope="module")
def system():
    rng = np.random.default_rng(0)
    q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    ev = np.linspace(0.0025, 1.0, N)  # condition number 400
    a = (q * ev) @ q.T
    b = rng.standard_normal(N)
    return a, b


def _classic(a, b, dt):
    """The engines' recurrence: alpha from <p, Ap>, beta from |r|^2."""
    ad = a.astype(dt)
    stop2 = TOL ** 2 * (b @ b)
    x_hi = np.zeros(N)
    x = np.zeros(N, dt)
    r_hi = b.copy()
    rho = r_hi @ r_hi
    r = r_hi.astype(dt)
    p = r.copy()
    rmax, it = np.sqrt(rho), 0
    while it < 5000:
        ap = ad @ p
        alpha = rho / float(p.astype(np.float64) @ ap.astype(np.float64))
        x = x + dt(alpha) * p
        r = r - dt(alpha) * ap
        t = float(r.astype(np.float64) @ r.astype(np.float64))
        it += 1
        rmax = max(rmax, np.sqrt(t))
        if t <= stop2 or np.sqrt(t) < DELTA * rmax:
            x_hi += x
            x[:] = 0
            r_hi = b - a @ x_hi
            t2 = r_hi @ r_hi
            if t2 <= stop2:
                return it, np.sqrt(t2 / (b @ b))
            beta, rho, rmax = t2 / rho, t2, np.sqrt(t2)
            r = r_hi.astype(dt)
            p = r + dt(beta) * p
            continue
        beta, rho = t / rho, t
        p = r + dt(beta) * p
    return it, None


def _pipelined(a, b, dt):
    """Ghysels-Vanroose: q = A w overlaps the reduction of |r|^2 and <w, r>;
    after an update w = A r is recomputed and s, z, p continue."""
    ad = a.astype(dt)
    stop2 = TOL ** 2 * (b @ b)
    x_hi = np.zeros(N)
    x = np.zeros(N, dt)
    p, s, z = (np.zeros(N, dt) for _ in range(3))
    r_hi = b.copy()
    rho = r_hi @ r_hi
    rmax, beta, alpha, it = np.sqrt(rho), 0.0, 0.0, 0
    r = r_hi.astype(dt)
    w = ad @ r
    restart = True
    while it < 5000:
        g = float(r.astype(np.float64) @ r.astype(np.float64))
        dl = float(w.astype(np.float64) @ r.astype(np.float64))
        if restart:
            restart, be = False, beta
        else:
            it += 1
            rmax = max(rmax, np.sqrt(g))
            if g <= stop2 or np.sqrt(g) < DELTA * rmax:
                x_hi += x
                x[:] = 0
                r_hi = b - a @ x_hi
                t2 = r_hi @ r_hi
                if t2 <= stop2:
                    return it, np.sqrt(t2 / (b @ b))
                beta, rho, rmax = t2 / rho, t2, np.sqrt(t2)
                r = r_hi.astype(dt)
                w = ad @ r
                restart = True
                continue
            be = g / rho
        pap = dl - (be * g / alpha if be != 0.0 else 0.0)
        alpha, rho = g / pap, g
        q = ad @ w
        z = q + dt(be) * z
        s = w + dt(be) * s
        p = r + dt(be) * p
        x = x + dt(alpha) * p
        r = r - dt(alpha) * s
        w = w - dt(alpha) * z
    return it, None


def test_pipelined_recurrence_needs_more_fp32_iterations(system):
    a, b = system
    it_c, res_c = _classic(a, b, np.float32)
    it_p, res_p = _pipelined(a, b, np.float32)
    assert res_c is not None and res_c <= TOL
    assert res_p is not None and res_p <= TOL
    assert it_p > 1.05 * it_c, (it_p, it_c)


def test_pipelined_recurrence_matches_in_fp64(system):
    a, b = system
    it_c, res_c = _classic(a, b, np.float64)
    it_p, res_p = _pipelined(a, b, np.float64)
    assert res_c <= TOL and res_p <= TOL
    assert abs(it_p - it_c) <= 0.03 * it_c + 2, (it_p, it_c)
