/*
 * Plain FP64 CPU oracle for the staggered Dirac operator, the even-odd
 * conjugate-gradient solve and the fermion force.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the HIP path against an obviously
 * correct reference.  It shares no code, header, table or helper with the HIP
 * path.
 *
 * What it follows.  The paper (Sec. 4) states that the framework provides a
 * staggered Dirac operator on SU(N) gauge links and single/double precision
 * conjugate-gradient solvers for it, on the 4-D grid of Sec. 1 with one SU(3)
 * matrix per link, and that hybrid Monte Carlo (whose molecular dynamics needs
 * the fermion force) is in progress.  It prints no formula, so the
 * definitions are the textbook Kogut-Susskind ones:
 *
 *   (D chi)(x) = 1/2 sum_mu eta_mu(x) [ bc_mu(x) U_mu(x) chi(x+mu)
 *                                      - bc_mu(x-mu) U_mu(x-mu)^dag chi(x-mu) ]
 *   eta_mu(x)  = (-1)^(x_0 + ... + x_{mu-1}),  mu = 0..3 = x, y, z, t
 *   bc_mu(x)   = -1 for mu = 3 and x_3 = L_3 - 1 when the antiperiodic-time
 *                flag is set, +1 otherwise; periodic wrap in every direction.
 *
 * With the Naik flag (the improved operator the paper's benchmark runs "with
 * and without the Naik term", Sec. 4) D gains a three-hop term and the
 * one-hop term is rescaled:
 *
 *   (D chi)(x) = 1/2 sum_mu eta_mu(x) { c1 [ bc U_mu(x) chi(x+mu) - (bc U_mu(x-mu))^dag chi(x-mu) ]
 *                                     + c3 [ N_mu(x) chi(x+3mu) - N_mu(x-3mu)^dag chi(x-3mu) ] }
 *   N_mu(x)    = (bc U_mu)(x) (bc U_mu)(x+mu) (bc U_mu)(x+2mu),  the parallel
 *                transporter along three links,
 *   c1 = 9/8, c3 = -1/24 (Naik's coefficients: the combination of the one- and
 *   three-step symmetric differences whose error starts at fifth order, so the
 *   free operator has sin p -> (9/8) sin p - (1/24) sin 3p).
 * The paper names the term but prints no coefficients or links; thin links in
 * both terms are this oracle's reading (no smearing).  eta_mu does not depend
 * on x_mu, so x and x +- 3 mu share it.
 *
 * D is anti-Hermitian.  D_eo (D_oe) is D with output restricted to even (odd)
 * sites and input to odd (even) sites.  The solver operator is
 * A = m^2 - D_eo D_oe on even sites, equal to (M^dag M) restricted to even
 * sites for M = m + D, hence Hermitian positive definite.
 *
 * Layouts are the plainest possible: lexicographic site order
 * lex = x0 + L0*(x1 + L1*(x2 + L2*x3)), array-of-structures, C99 double
 * complex.  U is [mu][lex][row][col]; a full-lattice colour vector is
 * [lex][colour]; a half-lattice vector of parity p holds the sites of parity p
 * in checkerboard order cb = lex >> 1 (valid because L0 is even).
 *
 * Parity status: every function here is pinned by tests against closed forms,
 * invariants or library routines; none is "parity unpinned".
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORACLE_BC_T_ANTIPERIODIC 1
#define ORACLE_NAIK 2

static const double NAIK_C1 = 9.0 / 8.0;
static const double NAIK_C3 = -1.0 / 24.0;

enum { ORACLE_OK = 0, ORACLE_NOTCONVERGED = 1, ORACLE_BREAKDOWN = 2, ORACLE_EINVAL = 3 };

/* ---------------------------------------------------------------- geometry */

static int64_t vol4(const int L[4]) {
  return (int64_t)L[0] * L[1] * L[2] * L[3];
}

static void coords_of(const int L[4], int64_t lex, int x[4]) {
  for (int mu = 0; mu < 4; ++mu) {
    x[mu] = (int)(lex % L[mu]);
    lex /= L[mu];
  }
}

static int64_t lex_of(const int L[4], const int x[4]) {
  return x[0] + (int64_t)L[0] * (x[1] + (int64_t)L[1] * (x[2] + (int64_t)L[2] * x[3]));
}

static int parity_of(const int x[4]) {
  return (x[0] + x[1] + x[2] + x[3]) & 1;
}

/* Staggered phase eta_mu(x) = (-1)^(sum_{nu < mu} x_nu). */
static double eta(int mu, const int x[4]) {
  int s = 0;
  for (int nu = 0; nu < mu; ++nu) s += x[nu];
  return (s & 1) ? -1.0 : 1.0;
}

/* Boundary sign carried by the link U_mu(x). */
static double bc_sign(const int L[4], int flags, int mu, const int x[4]) {
  if ((flags & ORACLE_BC_T_ANTIPERIODIC) && mu == 3 && x[3] == L[3] - 1) return -1.0;
  return 1.0;
}

static int dims_ok(const int L[4]) {
  for (int mu = 0; mu < 4; ++mu)
    if (L[mu] < 2 || (L[mu] & 1)) return 0;
  return 1;
}

/* Threads an OpenMP loop of the oracle runs on, and a way to change them
   (n >= 1; the timing of the CPU baseline on one core). */
int oracle_threads(void) { return omp_get_max_threads(); }
void oracle_set_threads(int n) { omp_set_num_threads(n >= 1 ? n : 1); }

/*
 * Even-odd index maps, for the bit-exact check of the device geometry.
 * eo = parity * V/2 + (lex >> 1).  lex_of_eo[eo] is the lexicographic site;
 * nbr_eo[8*eo + k] is the eo index of x + mu (k = mu) and x - mu (k = 4 + mu)
 * with periodic wrap.
 */

int oracle_index_maps(const int L[4], int32_t* lex_of_eo, int32_t* nbr_eo) {
  if (!dims_ok(L)) return ORACLE_EINVAL;
  const int64_t V = vol4(L), hv = V / 2;
  for (int64_t lex = 0; lex < V; ++lex) {
    int x[4];
    coords_of(L, lex, x);
    const int64_t eo = parity_of(x) * hv + (lex >> 1);
    lex_of_eo[eo] = (int32_t)lex;
    for (int mu = 0; mu < 4; ++mu) {
      for (int dir = 0; dir < 2; ++dir) {
        int y[4] = {x[0], x[1], x[2], x[3]};
        y[mu] = dir == 0 ? (x[mu] + 1) % L[mu] : (x[mu] - 1 + L[mu]) % L[mu];
        const int64_t ly = lex_of(L, y);
        nbr_eo[8 * eo + 4 * dir + mu] = (int32_t)(parity_of(y) * hv + (ly >> 1));
      }
    }
  }
  return ORACLE_OK;
}

/* ------------------------------------------------------------ Dirac operator */

static const cplx* link(const cplx* U, int64_t V, int mu, int64_t lex) {
  return U + ((int64_t)mu * V + lex) * 9;
}

/* N = (bc U_mu)(y) (bc U_mu)(y+mu) (bc U_mu)(y+2mu): the transporter from y+3mu to y. */
static void three_link(const int L[4], int flags, const cplx* U, int64_t V, int mu, const int y[4],
                       cplx N[9]) {
  int z[4] = {y[0], y[1], y[2], y[3]};
  cplx P[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  for (int step = 0; step < 3; ++step) {
    const cplx* Uz = link(U, V, mu, lex_of(L, z));
    const double s = bc_sign(L, flags, mu, z);
    cplx Q[9];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        cplx t = 0;
        for (int c = 0; c < 3; ++c) t += P[3 * a + c] * Uz[3 * c + b];
        Q[3 * a + b] = s * t;
      }
    memcpy(P, Q, sizeof P);
    z[mu] = (z[mu] + 1) % L[mu];
  }
  memcpy(N, P, sizeof P);
}

/* out = D in on the full lattice (both parities), with the factor 1/2. */
int oracle_dslash_full(const int L[4], int flags, const cplx* U, const cplx* in, cplx* out) {
  if (!dims_ok(L)) return ORACLE_EINVAL;
  const int64_t V = vol4(L);
  const int naik = flags & ORACLE_NAIK;
  const double c1 = naik ? NAIK_C1 : 1.0;
#pragma omp parallel for schedule(static)
  for (int64_t lex = 0; lex < V; ++lex) {
    int x[4];
    coords_of(L, lex, x);
    cplx acc[3] = {0, 0, 0};
    for (int mu = 0; mu < 4; ++mu) {
      int xp[4] = {x[0], x[1], x[2], x[3]};
      int xm[4] = {x[0], x[1], x[2], x[3]};
      xp[mu] = (x[mu] + 1) % L[mu];
      xm[mu] = (x[mu] - 1 + L[mu]) % L[mu];
      const int64_t lp = lex_of(L, xp), lm = lex_of(L, xm);
      const double ef = eta(mu, x) * bc_sign(L, flags, mu, x);
      const double eb = eta(mu, xm) * bc_sign(L, flags, mu, xm);
      const cplx* Uf = link(U, V, mu, lex); /* U_mu(x)    */
      const cplx* Ub = link(U, V, mu, lm);  /* U_mu(x-mu) */
      for (int a = 0; a < 3; ++a) {
        cplx fwd = 0, bwd = 0;
        for (int b = 0; b < 3; ++b) {
          fwd += Uf[3 * a + b] * in[3 * lp + b];
          bwd += conj(Ub[3 * b + a]) * in[3 * lm + b]; /* (U^dag)_{ab} = conj(U_{ba}) */
        }
        acc[a] += c1 * (ef * fwd - eb * bwd);
      }
      if (naik) {
        int x3p[4] = {x[0], x[1], x[2], x[3]};
        int x3m[4] = {x[0], x[1], x[2], x[3]};
        x3p[mu] = (x[mu] + 3) % L[mu];
        x3m[mu] = ((x[mu] - 3) % L[mu] + L[mu]) % L[mu];
        const int64_t l3p = lex_of(L, x3p), l3m = lex_of(L, x3m);
        cplx Nf[9], Nb[9];
        three_link(L, flags, U, V, mu, x, Nf);   /* N_mu(x)      */
        three_link(L, flags, U, V, mu, x3m, Nb); /* N_mu(x-3mu)  */
        const double e = eta(mu, x);
        for (int a = 0; a < 3; ++a) {
          cplx fwd = 0, bwd = 0;
          for (int b = 0; b < 3; ++b) {
            fwd += Nf[3 * a + b] * in[3 * l3p + b];
            bwd += conj(Nb[3 * b + a]) * in[3 * l3m + b];
          }
          acc[a] += NAIK_C3 * e * (fwd - bwd);
        }
      }
    }
    for (int a = 0; a < 3; ++a) out[3 * lex + a] = 0.5 * acc[a];
  }
  return ORACLE_OK;
}

/* Scatter a half-lattice vector of parity p into a zeroed full-lattice vector. */
static void scatter_half(const int L[4], int p, const cplx* half, cplx* full) {
  const int64_t V = vol4(L);
  memset(full, 0, sizeof(cplx) * 3 * V);
  for (int64_t lex = 0; lex < V; ++lex) {
    int x[4];
    coords_of(L, lex, x);
    if (parity_of(x) != p) continue;
    for (int a = 0; a < 3; ++a) full[3 * lex + a] = half[3 * (lex >> 1) + a];
  }
}

static void gather_half(const int L[4], int p, const cplx* full, cplx* half) {
  const int64_t V = vol4(L);
  for (int64_t lex = 0; lex < V; ++lex) {
    int x[4];
    coords_of(L, lex, x);
    if (parity_of(x) != p) continue;
    for (int a = 0; a < 3; ++a) half[3 * (lex >> 1) + a] = full[3 * lex + a];
  }
}

/*
 * Half-lattice operator: out (parity out_parity) = D in (parity 1-out_parity).
 * Computed as the full D restricted by parity masks, nothing cleverer.
 */
int oracle_dslash_eo(const int L[4], int flags, const cplx* U, int out_parity, const cplx* in_half,
                     cplx* out_half) {
  if (!dims_ok(L) || (out_parity != 0 && out_parity != 1)) return ORACLE_EINVAL;
  const int64_t V = vol4(L);
  cplx* fin = malloc(sizeof(cplx) * 3 * V);
  cplx* fout = malloc(sizeof(cplx) * 3 * V);
  if (!fin || !fout) {
    free(fin);
    free(fout);
    return ORACLE_EINVAL;
  }
  scatter_half(L, 1 - out_parity, in_half, fin);
  oracle_dslash_full(L, flags, U, fin, fout);
  gather_half(L, out_parity, fout, out_half);
  free(fin);
  free(fout);
  return ORACLE_OK;
}

/* out = A in = m^2 in - D_eo D_oe in, on even sites. */
int oracle_apply_A(const int L[4], int flags, const cplx* U, double mass, const cplx* in,
                   cplx* out) {
  if (!dims_ok(L)) return ORACLE_EINVAL;
  const int64_t hv = vol4(L) / 2;
  cplx* t = malloc(sizeof(cplx) * 3 * hv);
  cplx* s = malloc(sizeof(cplx) * 3 * hv);
  oracle_dslash_eo(L, flags, U, 1, in, t); /* t = D_oe in (odd)  */
  oracle_dslash_eo(L, flags, U, 0, t, s);  /* s = D_eo t  (even) */
  for (int64_t i = 0; i < 3 * hv; ++i) out[i] = mass * mass * in[i] - s[i];
  free(t);
  free(s);
  return ORACLE_OK;
}

/* ------------------------------------------------------------- CG (FP64) */

static double norm2(int64_t n, const cplx* v) {
  double s = 0;
  for (int64_t i = 0; i < n; ++i) s += creal(v[i]) * creal(v[i]) + cimag(v[i]) * cimag(v[i]);
  return s;
}

static double re_dot(int64_t n, const cplx* a, const cplx* b) {
  double s = 0;
  for (int64_t i = 0; i < n; ++i) s += creal(conj(a[i]) * b[i]);
  return s;
}

/*
 * Textbook Hestenes-Stiefel conjugate gradient for A x = b on even sites.
 * x holds the initial guess on entry when use_x0 is set, and the solution on
 * return.  Stops when the iterated residual satisfies |r| <= tol |b|, then
 * recomputes the true residual b - A x and, if that is still above tol |b|,
 * restarts from the current x.  Reports iterations and the true relative
 * residual.  Zero source gives x = 0 at once.
 */
int oracle_cg(const int L[4], int flags, const cplx* U, double mass, const cplx* b, cplx* x,
              int use_x0, double tol, int max_iter, int* iters_out, double* relres_out) {
  if (!dims_ok(L)) return ORACLE_EINVAL;
  const int64_t n = 3 * (vol4(L) / 2);
  cplx* r = malloc(sizeof(cplx) * n);
  cplx* p = malloc(sizeof(cplx) * n);
  cplx* Ap = malloc(sizeof(cplx) * n);
  if (!use_x0) memset(x, 0, sizeof(cplx) * n);
  const double bnorm = sqrt(norm2(n, b));
  int iters = 0, status = ORACLE_NOTCONVERGED;
  double relres = 0;
  if (bnorm == 0.0) {
    memset(x, 0, sizeof(cplx) * n);
    status = ORACLE_OK;
    goto done;
  }
  for (int restart = 0; restart < 100; ++restart) {
    oracle_apply_A(L, flags, U, mass, x, Ap);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - Ap[i];
    double rho = norm2(n, r);
    relres = sqrt(rho) / bnorm;
    if (relres <= tol) {
      status = ORACLE_OK;
      goto done;
    }
    memcpy(p, r, sizeof(cplx) * n);
    while (iters < max_iter) {
      oracle_apply_A(L, flags, U, mass, p, Ap);
      const double pAp = re_dot(n, p, Ap);
      if (!(pAp > 0.0) || !isfinite(pAp)) {
        status = ORACLE_BREAKDOWN;
        goto done;
      }
      const double alpha = rho / pAp;
      for (int64_t i = 0; i < n; ++i) {
        x[i] += alpha * p[i];
        r[i] -= alpha * Ap[i];
      }
      const double rho_new = norm2(n, r);
      ++iters;
      if (sqrt(rho_new) <= tol * bnorm) break;
      const double beta = rho_new / rho;
      for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
      rho = rho_new;
    }
    if (iters >= max_iter) {
      /* fall through to report the true residual of the last iterate */
      oracle_apply_A(L, flags, U, mass, x, Ap);
      for (int64_t i = 0; i < n; ++i) r[i] = b[i] - Ap[i];
      relres = sqrt(norm2(n, r)) / bnorm;
      status = relres <= tol ? ORACLE_OK : ORACLE_NOTCONVERGED;
      goto done;
    }
  }
done:
  if (iters_out) *iters_out = iters;
  if (relres_out) {
    if (bnorm == 0.0) {
      *relres_out = 0.0;
    } else {
      oracle_apply_A(L, flags, U, mass, x, Ap);
      for (int64_t i = 0; i < n; ++i) r[i] = b[i] - Ap[i];
      *relres_out = sqrt(norm2(n, r)) / bnorm;
    }
  }
  free(r);
  free(p);
  free(Ap);
  return status;
}

/* Relative true residual |b - A x| / |b| (0 for a zero source). */
double oracle_true_residual(const int L[4], int flags, const cplx* U, double mass, const cplx* b,
                            const cplx* x) {
  const int64_t n = 3 * (vol4(L) / 2);
  cplx* Ax = malloc(sizeof(cplx) * n);
  oracle_apply_A(L, flags, U, mass, x, Ax);
  double rr = 0;
  for (int64_t i = 0; i < n; ++i) {
    const cplx d = b[i] - Ax[i];
    rr += creal(d) * creal(d) + cimag(d) * cimag(d);
  }
  free(Ax);
  const double bn = sqrt(norm2(n, b));
  return bn == 0.0 ? sqrt(rr) : sqrt(rr) / bn;
}

/* ------------------------------------------- mixed precision, in emulation */

static double norm2_f(int64_t n, const float complex* v) {
  double s = 0;
  for (int64_t i = 0; i < n; ++i)
    s += (double)crealf(v[i]) * crealf(v[i]) + (double)cimagf(v[i]) * cimagf(v[i]);
  return s;
}

/*
 * Conjugate gradient with reliable updates (Sleijpen & van der Vorst 1996,
 * in the mixed-precision form of Clark et al., Comput. Phys. Commun. 181
 * (2010) 1517), in emulation: the iterated vectors x_lo, r, p, Ap are stored
 * in single precision (float complex) and A_lo applies the operator to a
 * single-precision vector with single-precision links, the dot products
 * accumulate in double.  The accumulated solution x_hi and the reliable
 * residual r_hi = b - A x_hi are double.  A reliable update happens when
 * |r| < delta * max|r| since the last one; convergence is only declared right
 * after a reliable update.  After an update p is kept and rho is taken from
 * r_hi.
 */
static void apply_A_single(const int L[4], int flags, const cplx* U_lo, double mass,
                           const float complex* in, float complex* out, cplx* tmp_in,
                           cplx* tmp_out, int64_t n) {
  /* Single-precision arithmetic is emulated by rounding the operands and the
     result to float; the products themselves run in double, which only makes
     the emulation slightly more accurate than true single precision. */
  for (int64_t i = 0; i < n; ++i) tmp_in[i] = in[i];
  oracle_apply_A(L, flags, U_lo, (double)(float)mass, tmp_in, tmp_out);
  for (int64_t i = 0; i < n; ++i) out[i] = (float complex)tmp_out[i];
}

int oracle_cg_mixed(const int L[4], int flags, const cplx* U, double mass, const cplx* b, cplx* x,
                    double tol, double delta, int max_iter, int* iters_out, int* updates_out,
                    double* relres_out) {
  if (!dims_ok(L)) return ORACLE_EINVAL;
  const int64_t V = vol4(L), n = 3 * (V / 2);
  cplx* U_lo = malloc(sizeof(cplx) * 36 * V);
  for (int64_t i = 0; i < 36 * V; ++i) U_lo[i] = (float complex)U[i];
  cplx* r_hi = malloc(sizeof(cplx) * n);
  cplx* t_in = malloc(sizeof(cplx) * n);
  cplx* t_out = malloc(sizeof(cplx) * n);
  float complex* r = malloc(sizeof(float complex) * n);
  float complex* p = malloc(sizeof(float complex) * n);
  float complex* Ap = malloc(sizeof(float complex) * n);
  float complex* x_lo = malloc(sizeof(float complex) * n);
  int iters = 0, updates = 0, status = ORACLE_NOTCONVERGED;
  const double bnorm = sqrt(norm2(n, b));
  memset(x, 0, sizeof(cplx) * n);
  if (bnorm == 0.0) {
    status = ORACLE_OK;
    goto done;
  }
  /* x_hi = 0, r_hi = b */
  memcpy(r_hi, b, sizeof(cplx) * n);
  for (int64_t i = 0; i < n; ++i) {
    r[i] = (float complex)r_hi[i];
    p[i] = r[i];
    x_lo[i] = 0;
  }
  double rho = norm2(n, r_hi);
  double rmax = sqrt(rho);
  while (iters < max_iter) {
    apply_A_single(L, flags, U_lo, mass, p, Ap, t_in, t_out, n);
    double pAp = 0;
    for (int64_t i = 0; i < n; ++i) pAp += creal(conj((cplx)p[i]) * (cplx)Ap[i]);
    if (!(pAp > 0.0) || !isfinite(pAp)) {
      status = ORACLE_BREAKDOWN;
      goto done;
    }
    const float alpha = (float)(rho / pAp);
    for (int64_t i = 0; i < n; ++i) {
      x_lo[i] += alpha * p[i];
      r[i] -= alpha * Ap[i];
    }
    double rho_new = norm2_f(n, r);
    ++iters;
    if (sqrt(rho_new) > rmax) rmax = sqrt(rho_new);
    const int converged_iterated = sqrt(rho_new) <= tol * bnorm;
    if (sqrt(rho_new) < delta * rmax || converged_iterated) {
      /* reliable update */
      for (int64_t i = 0; i < n; ++i) {
        x[i] += (cplx)x_lo[i];
        x_lo[i] = 0;
      }
      oracle_apply_A(L, flags, U, mass, x, t_out);
      for (int64_t i = 0; i < n; ++i) {
        r_hi[i] = b[i] - t_out[i];
        r[i] = (float complex)r_hi[i];
      }
      rho_new = norm2(n, r_hi);
      rmax = sqrt(rho_new);
      ++updates;
      if (sqrt(rho_new) <= tol * bnorm) {
        status = ORACLE_OK;
        goto done;
      }
    }
    const float beta = (float)(rho_new / rho);
    for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
    rho = rho_new;
  }
done:
  if (iters_out) *iters_out = iters;
  if (updates_out) *updates_out = updates;
  if (relres_out) *relres_out = bnorm == 0.0 ? 0.0 : oracle_true_residual(L, flags, U, mass, b, x);
  free(U_lo);
  free(r_hi);
  free(t_in);
  free(t_out);
  free(r);
  free(p);
  free(Ap);
  free(x_lo);
  return status;
}

/* ------------------------------------------------------------ fermion force */

/*
 * Gradient of a real function of the links, in the convention of PyTorch for
 * complex tensors: G = dF/dRe U + i dF/dIm U, one 3x3 matrix per link,
 * layout [mu][lex][row][col].
 *
 * For L(x) with x = A^{-1} b and upstream gradient g = dL/dRe x + i dL/dIm x,
 * let lam = A^{-1} g, y = D_oe x, nu = D_oe lam, and build the full-lattice
 * fields W1 = (lam on even, y on odd), W2 = (x on even, nu on odd).  Then
 *   G_mu(z) = 1/2 eps(z) eta_mu(z) bc_mu(z) [W1(z) W1(z+mu)^dag + W2(z) W2(z+mu)^dag]
 * with eps = +1 on even and -1 on odd sites.  This follows from
 * dx = -A^{-1} dA x and dA = -(dD_eo D_oe + D_eo dD_oe), using D_eo^dag = -D_oe.
 * For the action S = b^dag A^{-1} b one has g = b, lam = x and
 * G_mu(z) = eps eta bc w(z) w(z+mu)^dag with w = (x on even, y on odd).
 */
int oracle_force_from_fields(const int L[4], int flags, const cplx* U, const cplx* x_even,
                             const cplx* lam_even, cplx* G) {
  if (!dims_ok(L) || (flags & ORACLE_NAIK)) return ORACLE_EINVAL; /* one-hop operator only */
  const int64_t V = vol4(L), hv = V / 2;
  cplx* y = malloc(sizeof(cplx) * 3 * hv);
  cplx* nu = malloc(sizeof(cplx) * 3 * hv);
  cplx* W1 = malloc(sizeof(cplx) * 3 * V);
  cplx* W2 = malloc(sizeof(cplx) * 3 * V);
  oracle_dslash_eo(L, flags, U, 1, x_even, y);
  oracle_dslash_eo(L, flags, U, 1, lam_even, nu);
  for (int64_t lex = 0; lex < V; ++lex) {
    int xc[4];
    coords_of(L, lex, xc);
    const int64_t cb = lex >> 1;
    const int even = parity_of(xc) == 0;
    for (int a = 0; a < 3; ++a) {
      W1[3 * lex + a] = even ? lam_even[3 * cb + a] : y[3 * cb + a];
      W2[3 * lex + a] = even ? x_even[3 * cb + a] : nu[3 * cb + a];
    }
  }
#pragma omp parallel for schedule(static)
  for (int64_t lex = 0; lex < V; ++lex) {
    int z[4];
    coords_of(L, lex, z);
    const double eps = parity_of(z) == 0 ? 1.0 : -1.0;
    for (int mu = 0; mu < 4; ++mu) {
      int zp[4] = {z[0], z[1], z[2], z[3]};
      zp[mu] = (z[mu] + 1) % L[mu];
      const int64_t lp = lex_of(L, zp);
      const double s = 0.5 * eps * eta(mu, z) * bc_sign(L, flags, mu, z);
      cplx* g = G + ((int64_t)mu * V + lex) * 9;
      for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c)
          g[3 * a + c] = s * (W1[3 * lex + a] * conj(W1[3 * lp + c]) +
                              W2[3 * lex + a] * conj(W2[3 * lp + c]));
    }
  }
  free(y);
  free(nu);
  free(W1);
  free(W2);
  return ORACLE_OK;
}

/*
 * Action S = phi^dag A^{-1} phi (phi on even sites) and its link gradient.
 * x = A^{-1} phi by oracle_cg at the given tolerance.  x_out may be NULL.
 */
int oracle_force(const int L[4], int flags, const cplx* U, double mass, const cplx* phi,
                 double tol, int max_iter, cplx* G, double* S_out, cplx* x_out) {
  if (!dims_ok(L) || (flags & ORACLE_NAIK)) return ORACLE_EINVAL; /* one-hop operator only */
  const int64_t n = 3 * (vol4(L) / 2);
  cplx* x = malloc(sizeof(cplx) * n);
  int iters = 0;
  double rr = 0;
  const int st = oracle_cg(L, flags, U, mass, phi, x, 0, tol, max_iter, &iters, &rr);
  double S = 0;
  for (int64_t i = 0; i < n; ++i) S += creal(conj(phi[i]) * x[i]);
  if (S_out) *S_out = S;
  oracle_force_from_fields(L, flags, U, x, x, G);
  if (x_out) memcpy(x_out, x, sizeof(cplx) * n);
  free(x);
  return st;
}
