/*
 * oracle.c -- plain, slow, scalar FP64 reference for per-cell stiff chemistry.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle against which the GPU
 * library is checked.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the GPU library: it parses the mechanism text on its
 * own and recomputes everything from the definitions below.
 *
 * What it computes (the paper's problem statement, Sec. 3.1): in every cell,
 * advance the chemical state phi = (species, temperature) over one flow step
 * dt with an implicit (BDF) integrator whose Newton iteration uses the
 * chemical Jacobian J = d(rhs)/d(phi) (Eq. 7).  The chemistry itself:
 *   Eq. 1  mechanism  sum nu'_ij S_i <-> sum nu''_ij S_i
 *   Eq. 2  rate of progress Q_j = k_f,j prod C_i^nu'_ij - k_b,j prod C_i^nu''_ij
 *   Eq. 3  net production  wdot_i = sum_j (nu''_ij - nu'_ij) Q_j
 * The paper leaves the rate-constant forms, the energy equation, the BDF
 * variant and its error control unstated; the readings used here are:
 *   - k_f = exp(ln A + b ln T - (Ea/R)/T); K_c from Gibbs energies with
 *     p0 = 1 atm; k_b = k_f / K_c; third-body reactions multiply both
 *     directions by [M] = sum_k eps_k C_k (efficiencies 1 unless listed);
 *     Lindemann falloff k = k_inf Pr/(1+Pr), Pr = k_0 [M]/k_inf, optionally
 *     times Troe's broadening factor (CHEMKIN theory).
 *   - constant-pressure adiabatic reactor, state y = (Y_1..Y_S, T):
 *       dY_k/dt = W_k wdot_k / rho,  dT/dt = -sum_k H_k wdot_k / sum_k C_k Cp_k
 *   - species thermo with linear heat capacity cp/R = a0 + a1 T, or NASA
 *     7-coefficient polynomials in two temperature ranges.
 *   - quasi-constant-step BDF in backward-difference form, orders 1-5, a
 *     factored Newton matrix kept while recent (or fresh every step), WRMS
 *     error control, and after every accepted step projection of Y onto
 *     Y >= 0 (steps that would leave a mass fraction below -atol are
 *     rejected).
 * Units: the interface is SI (K, Pa, s, mass fractions); concentrations and
 * rate constants are cgs (mol/cm^3, A in mol-cm-s units).
 *
 * Build: gcc -O3 -std=c11 -fPIC -shared -fopenmp -ffp-contract=off
 * No fast-math and no FMA contraction, so every operation rounds as written.
 */
#include <ctype.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_SIDE 3

/* Physical constants (CODATA 2018 gas constant; thermochemical calorie). */
static const double ORC_RU = 8.31446261815324;      /* J/(mol K) */
static const double ORC_CAL = 4.184;                 /* J/cal */
static const double ORC_PATM = 101325.0;             /* Pa, standard-state pressure */
static const double ORC_TREF = 298.15;               /* K, thermo reference */

#define ORC_MAX_EFF 32

typedef struct {
  int rev, type;             /* type 0 elementary, 1 third body, 2 falloff (Lindemann, or Troe when ntroe > 0) */
  int nr, np;
  int r[ORC_MAX_SIDE], p[ORC_MAX_SIDE];
  double A, b, Ea_kcal;
  double A0, b0, Ea0_kcal;   /* falloff low-pressure limit */
  int ntroe;                 /* 0, or 3/4 Troe parameters alpha, T3, T1 [, T2] (CHEMKIN's T***, T*, T**) */
  double troe[4];
  int neff;                  /* collision efficiencies other than 1 in [M] */
  int effk[ORC_MAX_EFF];
  double effv[ORC_MAX_EFF];
  int drop_f, drop_r;        /* direction removed by the one-sided linearisation of QSS couplings */
} orc_reaction;

typedef struct {
  int E, S, R;
  double emass[8];
  int *atoms;                /* [S][E] */
  int *inert;
  double *W, *a0, *a1, *hf, *s0;
  int *nasa;                 /* [S] 1: NASA 7-coefficient thermo (nasa_c), 0: linear cp (a0, a1, hf, s0) */
  double *nasa_c;            /* [S][15]: T_mid, 7 coefficients for T <= T_mid, 7 for T > T_mid */
  orc_reaction *rx;
  int *nu;                   /* [S][R] net stoichiometric coefficient nu'' - nu' */
  /* quasi-steady-state species (Sec. 2.1): nq of them, algebraic; the state
   * holds the ST = S - nq transported species */
  int nq, ST;
  int *isq;                  /* [S] position among the QSS species, or -1 */
  int *tsp;                  /* [ST] species of state component i */
  int *qsp;                  /* [nq] species of QSS unknown q */
} orc_mech;

/* --------------------------------------------------------------- parsing -- */

typedef struct { const char *s; } orc_lex;

static int orc_next(orc_lex *L, char *tok, int cap) {
  for (;;) {
    while (*L->s && isspace((unsigned char)*L->s)) L->s++;
    if (*L->s == '#') { while (*L->s && *L->s != '\n') L->s++; continue; }
    break;
  }
  if (!*L->s) return 0;
  int n = 0;
  while (*L->s && !isspace((unsigned char)*L->s) && *L->s != '#') {
    if (n < cap - 1) tok[n++] = *L->s;
    L->s++;
  }
  tok[n] = 0;
  return 1;
}

static int orc_int(orc_lex *L, int *v) {
  char t[128], *e;
  if (!orc_next(L, t, sizeof t)) return 0;
  long x = strtol(t, &e, 10);
  if (*e) return 0;
  *v = (int)x;
  return 1;
}

static int orc_dbl(orc_lex *L, double *v) {
  char t[128], *e;
  if (!orc_next(L, t, sizeof t)) return 0;
  *v = strtod(t, &e);
  return *e == 0 && isfinite(*v);
}

static int orc_word(orc_lex *L, const char *w) {
  char t[128];
  return orc_next(L, t, sizeof t) && strcmp(t, w) == 0;
}

/* True (and the word consumed) when the next token is w; otherwise nothing is consumed. */
static int orc_opt_word(orc_lex *L, const char *w) {
  orc_lex save = *L;
  char t[128];
  if (orc_next(L, t, sizeof t) && strcmp(t, w) == 0) return 1;
  *L = save;
  return 0;
}

void orc_free(orc_mech *m) {
  if (!m) return;
  free(m->atoms); free(m->inert); free(m->W); free(m->a0); free(m->a1);
  free(m->hf); free(m->s0); free(m->nasa); free(m->nasa_c); free(m->rx); free(m->nu);
  free(m->isq); free(m->tsp); free(m->qsp); free(m);
}

/* Parse the mechanism text (format documented with the generator) and derive
 * molecular weights W_k = sum_e n_ek m_e and the net coefficients of Eq. 3. */
orc_mech *orc_load(const char *text, char *err, int errlen) {
  orc_lex L = {text};
  char name[128];
  orc_mech *m = calloc(1, sizeof *m);
#define FAIL(msg) do { if (err) snprintf(err, errlen, "%s", msg); orc_free(m); return NULL; } while (0)
  if (!orc_word(&L, "chem-mech")) FAIL("missing header");
  int ver;
  if (!orc_int(&L, &ver) || ver != 1) FAIL("bad version");
  if (!orc_word(&L, "ELEMENTS") || !orc_int(&L, &m->E) || m->E < 1 || m->E > 8) FAIL("bad ELEMENTS");
  for (int e = 0; e < m->E; ++e)
    if (!orc_next(&L, name, sizeof name) || !orc_dbl(&L, &m->emass[e]) || m->emass[e] <= 0) FAIL("bad element");
  if (!orc_word(&L, "SPECIES") || !orc_int(&L, &m->S) || m->S < 1 || m->S > 1024) FAIL("bad SPECIES");
  int S = m->S, E = m->E;
  m->atoms = calloc((size_t)S * E, sizeof(int));
  m->inert = calloc(S, sizeof(int));
  m->W = calloc(S, sizeof(double)); m->a0 = calloc(S, sizeof(double));
  m->a1 = calloc(S, sizeof(double)); m->hf = calloc(S, sizeof(double));
  m->s0 = calloc(S, sizeof(double));
  m->nasa = calloc(S, sizeof(int));
  m->nasa_c = calloc((size_t)S * 15, sizeof(double));
  for (int k = 0; k < S; ++k) {
    if (!orc_next(&L, name, sizeof name) || !orc_int(&L, &m->inert[k])) FAIL("bad species line");
    double W = 0.0;
    int tot = 0;
    for (int e = 0; e < E; ++e) {
      if (!orc_int(&L, &m->atoms[k * E + e]) || m->atoms[k * E + e] < 0) FAIL("bad atom count");
      W += m->atoms[k * E + e] * m->emass[e];
      tot += m->atoms[k * E + e];
    }
    if (tot == 0) FAIL("species without atoms");
    m->W[k] = W;
    if (orc_opt_word(&L, "NASA7")) {
      m->nasa[k] = 1;
      for (int i = 0; i < 15; ++i)
        if (!orc_dbl(&L, &m->nasa_c[k * 15 + i])) FAIL("bad NASA7 thermo");
      if (!(m->nasa_c[k * 15] > 0)) FAIL("bad NASA7 midpoint temperature");
    } else if (!orc_dbl(&L, &m->a0[k]) || !orc_dbl(&L, &m->a1[k]) || !orc_dbl(&L, &m->hf[k]) ||
               !orc_dbl(&L, &m->s0[k])) {
      FAIL("bad thermo");
    }
  }
  if (!orc_word(&L, "REACTIONS") || !orc_int(&L, &m->R) || m->R < 0 || m->R > 100000) FAIL("bad REACTIONS");
  int R = m->R;
  m->rx = calloc(R > 0 ? R : 1, sizeof(orc_reaction));
  m->nu = calloc((size_t)S * (R > 0 ? R : 1), sizeof(int));
  for (int j = 0; j < R; ++j) {
    orc_reaction *x = &m->rx[j];
    if (!orc_int(&L, &x->rev) || !orc_int(&L, &x->type) || x->type < 0 || x->type > 2) FAIL("bad reaction kind");
    if (!orc_int(&L, &x->nr) || x->nr < 1 || x->nr > ORC_MAX_SIDE) FAIL("bad reactant count");
    for (int i = 0; i < x->nr; ++i)
      if (!orc_int(&L, &x->r[i]) || x->r[i] < 0 || x->r[i] >= S) FAIL("bad reactant index");
    if (!orc_int(&L, &x->np) || x->np < 1 || x->np > ORC_MAX_SIDE) FAIL("bad product count");
    for (int i = 0; i < x->np; ++i)
      if (!orc_int(&L, &x->p[i]) || x->p[i] < 0 || x->p[i] >= S) FAIL("bad product index");
    if (!orc_dbl(&L, &x->A) || !orc_dbl(&L, &x->b) || !orc_dbl(&L, &x->Ea_kcal) || x->A <= 0) FAIL("bad Arrhenius");
    if (x->type == 2 && (!orc_dbl(&L, &x->A0) || !orc_dbl(&L, &x->b0) || !orc_dbl(&L, &x->Ea0_kcal) || x->A0 <= 0))
      FAIL("bad falloff");
    if (orc_opt_word(&L, "TROE")) {
      if (x->type != 2 || !orc_int(&L, &x->ntroe) || (x->ntroe != 3 && x->ntroe != 4)) FAIL("bad TROE");
      for (int i = 0; i < x->ntroe; ++i)
        if (!orc_dbl(&L, &x->troe[i])) FAIL("bad TROE parameter");
      if (x->troe[1] == 0.0 || x->troe[2] == 0.0) FAIL("TROE temperatures T3 and T1 must be nonzero");
    }
    if (orc_opt_word(&L, "EFF")) {
      if (x->type == 0 || !orc_int(&L, &x->neff) || x->neff < 0 || x->neff > ORC_MAX_EFF) FAIL("bad EFF");
      for (int i = 0; i < x->neff; ++i) {
        if (!orc_int(&L, &x->effk[i]) || x->effk[i] < 0 || x->effk[i] >= S || !orc_dbl(&L, &x->effv[i]) ||
            x->effv[i] < 0)
          FAIL("bad efficiency");
        for (int i2 = 0; i2 < i; ++i2)
          if (x->effk[i2] == x->effk[i]) FAIL("repeated efficiency");
      }
    }
    for (int i = 0; i < x->nr; ++i) m->nu[x->r[i] * R + j] -= 1;
    for (int i = 0; i < x->np; ++i) m->nu[x->p[i] * R + j] += 1;
    for (int e = 0; e < E; ++e) {   /* element balance, exact in integers */
      int bal = 0;
      for (int k = 0; k < S; ++k) bal += m->nu[k * R + j] * m->atoms[k * E + e];
      if (bal != 0) FAIL("reaction not atom balanced");
    }
  }
  /* optional QSS record: the species the quasi-steady-state approximation
   * (Eq. 4) turns into algebraic unknowns */
  m->isq = malloc(sizeof(int) * S);
  for (int k = 0; k < S; ++k) m->isq[k] = -1;
  if (orc_opt_word(&L, "QSS")) {
    if (!orc_int(&L, &m->nq) || m->nq < 0 || m->nq >= S) FAIL("bad QSS record");
    m->qsp = malloc(sizeof(int) * (m->nq > 0 ? m->nq : 1));
    for (int q = 0; q < m->nq; ++q) {
      int k;
      if (!orc_int(&L, &k) || k < 0 || k >= S || m->isq[k] >= 0 || m->inert[k]) FAIL("bad QSS species");
      m->qsp[q] = k;
      m->isq[k] = q;
    }
  } else {
    m->qsp = malloc(sizeof(int));
  }
  m->ST = S - m->nq;
  m->tsp = malloc(sizeof(int) * m->ST);
  for (int k = 0, i = 0; k < S; ++k)
    if (m->isq[k] < 0) m->tsp[i++] = k;
  /* one-sided linearisation (Sec. 2.2): a direction with two or more QSS
   * species among its reactants would make the closure nonlinear and is
   * removed; the other direction of the reaction stays */
  for (int j = 0; j < R; ++j) {
    orc_reaction *x = &m->rx[j];
    int nqr = 0, nqp = 0;
    for (int i = 0; i < x->nr; ++i) nqr += m->isq[x->r[i]] >= 0;
    for (int i = 0; i < x->np; ++i) nqp += m->isq[x->p[i]] >= 0;
    x->drop_f = nqr >= 2;
    x->drop_r = nqp >= 2;
  }
  /* every QSS species must be consumed by a kept direction, or its closure
   * equation has no diagonal term */
  for (int q = 0; q < m->nq; ++q) {
    int k = m->qsp[q], consumed = 0;
    for (int j = 0; j < R; ++j) {
      const orc_reaction *x = &m->rx[j];
      int n = m->nu[k * R + j], inr = 0, inp = 0;
      for (int i = 0; i < x->nr; ++i) inr |= x->r[i] == k;
      for (int i = 0; i < x->np; ++i) inp |= x->p[i] == k;
      if ((n < 0 && inr && !x->drop_f) || (n > 0 && inp && x->rev && !x->drop_r)) consumed = 1;
    }
    if (!consumed) FAIL("a QSS species is never consumed");
  }
  if (!orc_word(&L, "END")) FAIL("missing END");
#undef FAIL
  return m;
}

int orc_qss_info(const orc_mech *m, int *nq, int *qsp) {
  *nq = m->nq;
  if (qsp) for (int q = 0; q < m->nq; ++q) qsp[q] = m->qsp[q];
  return m->ST;
}

int orc_info(const orc_mech *m, int *S, int *R, int *E) {
  *S = m->S; *R = m->R; *E = m->E;
  return 0;
}

void orc_weights(const orc_mech *m, double *W) { for (int k = 0; k < m->S; ++k) W[k] = m->W[k]; }

int orc_nu(const orc_mech *m, int *nu) { memcpy(nu, m->nu, sizeof(int) * m->S * m->R); return 0; }

/* ---------------------------------------------------------------- thermo -- */

/* Molar enthalpy, entropy, heat capacity and its T-derivative of species k
 * (J/mol, J/(mol K), J/(mol K^2)).
 *   linear:  cp/R = a0 + a1 T, integrated from h_f and s0 at 298.15 K;
 *   NASA 7-coefficient polynomials (the CHEMKIN thermo form of real
 *   mechanisms), coefficients c1..c7 of the range holding T (T <= T_mid: the
 *   low range):
 *     cp/R = c1 + c2 T + c3 T^2 + c4 T^3 + c5 T^4
 *     H/(R T) = c1 + c2 T/2 + c3 T^2/3 + c4 T^3/4 + c5 T^4/5 + c6/T
 *     S/R = c1 ln T + c2 T + c3 T^2/2 + c4 T^3/3 + c5 T^4/4 + c7 */
static void orc_species_thermo(const orc_mech *m, int k, double T, double *h, double *s, double *cp, double *dcp) {
  if (m->nasa[k]) {
    const double *c = m->nasa_c + (size_t)k * 15;
    const double *a = T <= c[0] ? c + 1 : c + 8;
    double T2 = T * T, T3 = T2 * T, T4 = T3 * T;
    *cp = ORC_RU * (a[0] + a[1] * T + a[2] * T2 + a[3] * T3 + a[4] * T4);
    *h = ORC_RU * (a[0] * T + a[1] * T2 / 2.0 + a[2] * T3 / 3.0 + a[3] * T4 / 4.0 + a[4] * T4 * T / 5.0 + a[5]);
    *s = ORC_RU * (a[0] * log(T) + a[1] * T + a[2] * T2 / 2.0 + a[3] * T3 / 3.0 + a[4] * T4 / 4.0 + a[6]);
    *dcp = ORC_RU * (a[1] + 2.0 * a[2] * T + 3.0 * a[3] * T2 + 4.0 * a[4] * T3);
    return;
  }
  double a0 = m->a0[k], a1 = m->a1[k];
  *h = m->hf[k] + ORC_RU * (a0 * (T - ORC_TREF) + a1 * (T * T - ORC_TREF * ORC_TREF) / 2.0);
  *s = m->s0[k] + ORC_RU * (a0 * log(T / ORC_TREF) + a1 * (T - ORC_TREF));
  *cp = ORC_RU * (a0 + a1 * T);
  *dcp = ORC_RU * a1;
}

/* Per-species molar enthalpy, entropy, heat capacity and Gibbs energy (J/mol,
 * J/(mol K)). */
void orc_thermo(const orc_mech *m, double T, double *H, double *Sm, double *Cp, double *G) {
  for (int k = 0; k < m->S; ++k) {
    double h, s, cp, dcp;
    orc_species_thermo(m, k, T, &h, &s, &cp, &dcp);
    if (H) H[k] = h;
    if (Sm) Sm[k] = s;
    if (Cp) Cp[k] = cp;
    if (G) G[k] = h - T * s;
  }
}

/* d Cp_k / dT for every species (J/(mol K^2)). */
void orc_dcp_dT(const orc_mech *m, double T, double *dCp) {
  for (int k = 0; k < m->S; ++k) {
    double h, s, cp;
    orc_species_thermo(m, k, T, &h, &s, &cp, &dCp[k]);
  }
}

/* Third-body concentration of reaction j: [M]_j = sum_k eps_jk C_k, with
 * eps = 1 except where the reaction lists another efficiency. */
static double orc_third_body(const orc_mech *m, int j, const double *C, double Mconc) {
  const orc_reaction *x = &m->rx[j];
  double M = Mconc;
  for (int i = 0; i < x->neff; ++i)
    if (m->isq[x->effk[i]] < 0) M += (x->effv[i] - 1.0) * C[x->effk[i]];
  return M;
}

/* d[M]_j / dC_c.  QSS species are not colliders: [M] sums the transported
 * species only. */
static double orc_efficiency(const orc_mech *m, const orc_reaction *x, int c) {
  if (m->isq[c] >= 0) return 0.0;
  for (int i = 0; i < x->neff; ++i)
    if (x->effk[i] == c) return x->effv[i];
  return 1.0;
}

/* Mixture: mean molecular weight, density (g/cm^3) and concentrations (mol/cm^3). */
static void orc_mixture(const orc_mech *m, double T, const double *Y, double p, double *rho, double *Wbar, double *C) {
  double inv = 0.0;
  for (int k = 0; k < m->S; ++k) inv += Y[k] / m->W[k];
  double Wb = 1.0 / inv;
  double r = (p * 10.0) * Wb / (ORC_RU * 1.0e7 * T);   /* dyn/cm^2 * g/mol / (erg/mol/K * K) */
  for (int k = 0; k < m->S; ++k) C[k] = r * Y[k] / m->W[k];
  *rho = r;
  *Wbar = Wb;
}

/* ----------------------------------------------------------------- rates -- */

/* Rate constants of reaction j (Eq. 2's k vector) and their T-derivatives at
 * fixed concentrations.  G_RT[k] = G_k/(R T), H[k] in J/mol, Mconc = [M]. */
typedef struct { double kf, kr, dkf, dkr, dkf_dM, dkr_dM; } orc_k;

static orc_k orc_rate_constants(const orc_mech *m, int j, double T, const double *G, const double *H, double Mconc) {
  const orc_reaction *x = &m->rx[j];
  orc_k K = {0, 0, 0, 0, 0, 0};
  double EaR = x->Ea_kcal * 1000.0 * ORC_CAL / ORC_RU;          /* K */
  double kinf = exp(log(x->A) + x->b * log(T) - EaR / T);
  double dlnkinf = (x->b + EaR / T) / T;
  double kf = kinf, dlnkf = dlnkinf, dkf_dM = 0.0;
  if (x->type == 2) {
    double EaR0 = x->Ea0_kcal * 1000.0 * ORC_CAL / ORC_RU;
    double k0 = exp(log(x->A0) + x->b0 * log(T) - EaR0 / T);
    double dlnk0 = (x->b0 + EaR0 / T) / T;
    double Pr = k0 * Mconc / kinf;
    kf = kinf * Pr / (1.0 + Pr);
    /* d ln kf/dT = d ln kinf/dT + (d ln Pr/dT)/(1+Pr), d ln Pr/dT = d ln k0 - d ln kinf */
    dlnkf = dlnkinf + (dlnk0 - dlnkinf) / (1.0 + Pr);
    dkf_dM = k0 / ((1.0 + Pr) * (1.0 + Pr));
    if (x->ntroe) {
      /* Troe's broadening factor (CHEMKIN form), logarithms base 10:
       *   F_cent = (1-a) exp(-T/T3) + a exp(-T/T1) [+ exp(-T2/T)]
       * (T3, T1, T2 are CHEMKIN's T***, T* and T**)
       *   c = -0.4 - 0.67 log F_cent,  n = 0.75 - 1.27 log F_cent,  d = 0.14
       *   f1 = (log Pr + c) / (n - d (log Pr + c))
       *   log F = log F_cent / (1 + f1^2),   k = k_inf Pr/(1+Pr) F
       * with log Pr taken at max(Pr, 1e-300) so that [M] = 0 stays finite. */
      const double a = x->troe[0], T3 = x->troe[1], T1 = x->troe[2];
      double Fc = (1.0 - a) * exp(-T / T3) + a * exp(-T / T1);
      double dFc = -(1.0 - a) / T3 * exp(-T / T3) - a / T1 * exp(-T / T1);
      if (x->ntroe == 4) {
        const double T2 = x->troe[3];
        Fc += exp(-T2 / T);
        dFc += T2 / (T * T) * exp(-T2 / T);
      }
      const double ln10 = log(10.0);
      double Lc = log10(Fc);
      double lp = log10(Pr > 1e-300 ? Pr : 1e-300);
      double cc = -0.4 - 0.67 * Lc, nn = 0.75 - 1.27 * Lc, dd = 0.14;
      double u = lp + cc, v = nn - dd * u;
      double f1 = u / v;
      double den = 1.0 + f1 * f1;
      double logF = Lc / den;
      double F = pow(10.0, logF);
      /* partial derivatives of log F: in log Pr (L_c fixed) and in L_c (log Pr fixed) */
      double df1_dlp = nn / (v * v);
      double df1_dLc = (-0.67 * v - u * (-1.27 + 0.67 * dd)) / (v * v);
      double dlogF_dlp = -Lc * 2.0 * f1 * df1_dlp / (den * den);
      double dlogF_dLc = 1.0 / den - Lc * 2.0 * f1 * df1_dLc / (den * den);
      double dLc_dT = dFc / (Fc * ln10);
      double dlp_dT = (Pr > 1e-300) ? (dlnk0 - dlnkinf) / ln10 : 0.0;
      double dlnF_dT = ln10 * (dlogF_dlp * dlp_dT + dlogF_dLc * dLc_dT);
      /* d F/d[M] = F ln10 dlogF/dlp d lp/d[M] = F dlogF/dlp / [M]; times kinf Pr/(1+Pr) = k0 [M]/(1+Pr) */
      dkf_dM = F * dkf_dM + F * k0 / (1.0 + Pr) * (Pr > 1e-300 ? dlogF_dlp : 0.0);
      kf *= F;
      dlnkf += dlnF_dT;
    }
  }
  K.kf = kf;
  K.dkf = kf * dlnkf;
  K.dkf_dM = dkf_dM;
  if (x->rev) {
    /* K_c = exp(-sum_k nu_kj G_k/RT) (p0/(R T))^dnu, p0/(RT) in mol/cm^3 */
    double sumG = 0.0, sumH = 0.0;
    int dnu = 0;
    for (int k = 0; k < m->S; ++k) {
      int n = m->nu[k * m->R + j];
      if (n) { sumG += n * G[k]; sumH += n * H[k]; dnu += n; }
    }
    double c0 = ORC_PATM / (ORC_RU * T) * 1.0e-6;
    double Kc = exp(-sumG) * pow(c0, (double)dnu);
    /* d ln Kc/dT = sum nu H/(R T^2) - dnu/T (van 't Hoff plus the c0 factor) */
    double dlnKc = sumH / (ORC_RU * T * T) - dnu / T;
    K.kr = kf / Kc;
    K.dkr = K.kr * (dlnkf - dlnKc);
    K.dkr_dM = dkf_dM / Kc;
  }
  return K;
}

/* Per-reaction rate constants and rates of progress (Eq. 2), and net
 * production rates (Eq. 3), for one cell.  Outputs may be NULL. */
int orc_rates(const orc_mech *m, double T, const double *Y, double p, double *kf, double *kr, double *Q, double *wdot) {
  int S = m->S, R = m->R;
  double *C = malloc(sizeof(double) * S * 4);
  double *H = C + S, *G = C + 2 * S, *Sm = C + 3 * S;
  double rho, Wbar;
  orc_mixture(m, T, Y, p, &rho, &Wbar, C);
  orc_thermo(m, T, H, Sm, NULL, G);
  for (int k = 0; k < S; ++k) G[k] /= ORC_RU * T;
  double Mconc = 0.0;
  for (int k = 0; k < S; ++k) Mconc += C[k];
  if (wdot) for (int k = 0; k < S; ++k) wdot[k] = 0.0;
  for (int j = 0; j < R; ++j) {
    const orc_reaction *x = &m->rx[j];
    double Mj = orc_third_body(m, j, C, Mconc);
    orc_k K = orc_rate_constants(m, j, T, G, H, Mj);
    double pf = 1.0, pr = 1.0;
    for (int i = 0; i < x->nr; ++i) pf *= C[x->r[i]];
    for (int i = 0; i < x->np; ++i) pr *= C[x->p[i]];
    double q = K.kf * pf - K.kr * pr;
    if (x->type == 1) q *= Mj;
    if (kf) kf[j] = K.kf;
    if (kr) kr[j] = K.kr;
    if (Q) Q[j] = q;
    if (wdot) for (int k = 0; k < S; ++k) wdot[k] += m->nu[k * R + j] * q;
  }
  free(C);
  return 0;
}

/* ------------------------------------------------------------- ODE system -- */

static int orc_rhs_qss(const orc_mech *m, const double *y, double p, int fixed_T, double *f);
static int orc_jac_qss(const orc_mech *m, const double *y, double p, int fixed_T, double *J);

/* Right-hand side of the constant-pressure adiabatic reactor, y = (Y, T). */
int orc_rhs(const orc_mech *m, const double *y, double p, int fixed_T, double *f) {
  if (m->nq) return orc_rhs_qss(m, y, p, fixed_T, f);
  int S = m->S;
  double T = y[S];
  double *C = malloc(sizeof(double) * S * 4);
  double *H = C + S, *Cp = C + 2 * S, *wd = C + 3 * S;
  double rho, Wbar;
  orc_mixture(m, T, y, p, &rho, &Wbar, C);
  orc_thermo(m, T, H, NULL, Cp, NULL);
  orc_rates(m, T, y, p, NULL, NULL, NULL, wd);
  double num = 0.0, den = 0.0;
  for (int k = 0; k < S; ++k) {
    f[k] = m->W[k] * wd[k] / rho;
    num += H[k] * wd[k];
    den += C[k] * Cp[k];
  }
  f[S] = fixed_T ? 0.0 : -num / den;
  free(C);
  return 0;
}

/* Analytic Jacobian J[i][j] = d f_i / d y_j (row-major, N = S+1), Eq. 7 in
 * the state (Y, T).  First the concentration-space Jacobian A = d wdot/dC and
 * b = d wdot/dT at fixed C are accumulated reaction by reaction, then the chain
 * rule through C_k(Y, T) and rho(Y, T) is applied as plain dense products. */
int orc_jac(const orc_mech *m, const double *y, double p, int fixed_T, double *J) {
  if (m->nq) return orc_jac_qss(m, y, p, fixed_T, J);
  int S = m->S, R = m->R, N = S + 1;
  double T = y[S];
  double *C = malloc(sizeof(double) * (size_t)(8 * S + S * S + 2 * S * N + N));
  double *H = C + S, *Cp = H + S, *G = Cp + S, *Sm = G + S, *wd = Sm + S, *b = wd + S, *dCp = b + S;
  double *A = dCp + S;              /* [S][S] */
  double *dC = A + S * S;           /* [S][N]: dC_m/dy_j */
  double *dw = dC + S * N;          /* [S][N]: d wdot_k/dy_j */
  double *drho = dw + S * N;        /* [N] */
  double rho, Wbar;
  orc_mixture(m, T, y, p, &rho, &Wbar, C);
  orc_thermo(m, T, H, Sm, Cp, G);
  orc_dcp_dT(m, T, dCp);
  for (int k = 0; k < S; ++k) G[k] /= ORC_RU * T;
  double Mconc = 0.0;
  for (int k = 0; k < S; ++k) Mconc += C[k];
  for (int i = 0; i < S * S; ++i) A[i] = 0.0;
  for (int k = 0; k < S; ++k) { b[k] = 0.0; wd[k] = 0.0; }
  for (int j = 0; j < R; ++j) {
    const orc_reaction *x = &m->rx[j];
    double Mj = orc_third_body(m, j, C, Mconc);
    orc_k K = orc_rate_constants(m, j, T, G, H, Mj);
    double pf = 1.0, pr = 1.0;
    for (int i = 0; i < x->nr; ++i) pf *= C[x->r[i]];
    for (int i = 0; i < x->np; ++i) pr *= C[x->p[i]];
    double mfac = (x->type == 1) ? Mj : 1.0;
    double q = mfac * (K.kf * pf - K.kr * pr);
    double dq_dT = mfac * (K.dkf * pf - K.dkr * pr);
    /* dq/dC_c for every species c: product rule over the reactant/product lists */
    for (int c = 0; c < S; ++c) {
      double dpf = 0.0, dpr = 0.0;
      for (int i = 0; i < x->nr; ++i) {
        if (x->r[i] != c) continue;
        double t = 1.0;
        for (int i2 = 0; i2 < x->nr; ++i2) if (i2 != i) t *= C[x->r[i2]];
        dpf += t;
      }
      for (int i = 0; i < x->np; ++i) {
        if (x->p[i] != c) continue;
        double t = 1.0;
        for (int i2 = 0; i2 < x->np; ++i2) if (i2 != i) t *= C[x->p[i2]];
        dpr += t;
      }
      double dq = mfac * (K.kf * dpf - K.kr * dpr);
      double eps = (x->type == 0) ? 0.0 : orc_efficiency(m, x, c);   /* d[M]_j/dC_c */
      if (x->type == 1) dq += eps * (K.kf * pf - K.kr * pr);
      if (x->type == 2) dq += eps * (K.dkf_dM * pf - K.dkr_dM * pr);
      for (int k = 0; k < S; ++k) A[k * S + c] += m->nu[k * R + j] * dq;
    }
    for (int k = 0; k < S; ++k) {
      b[k] += m->nu[k * R + j] * dq_dT;
      wd[k] += m->nu[k * R + j] * q;
    }
  }
  /* dC_m/dY_j = delta_mj rho/W_m - C_m Wbar/W_j ; dC_m/dT = -C_m/T */
  for (int mm = 0; mm < S; ++mm) {
    for (int j = 0; j < S; ++j) dC[mm * N + j] = (mm == j ? rho / m->W[mm] : 0.0) - C[mm] * Wbar / m->W[j];
    dC[mm * N + S] = -C[mm] / T;
  }
  for (int j = 0; j < S; ++j) drho[j] = -rho * Wbar / m->W[j];
  drho[S] = -rho / T;
  for (int k = 0; k < S; ++k)
    for (int j = 0; j < N; ++j) {
      double s = 0.0;
      for (int mm = 0; mm < S; ++mm) s += A[k * S + mm] * dC[mm * N + j];
      if (j == S) s += b[k];
      dw[k * N + j] = s;
    }
  /* species rows: f_k = W_k wdot_k / rho */
  for (int k = 0; k < S; ++k)
    for (int j = 0; j < N; ++j)
      J[k * N + j] = m->W[k] / rho * dw[k * N + j] - m->W[k] * wd[k] / (rho * rho) * drho[j];
  /* temperature row: f_T = -num/den */
  double num = 0.0, den = 0.0;
  for (int k = 0; k < S; ++k) { num += H[k] * wd[k]; den += C[k] * Cp[k]; }
  for (int j = 0; j < N; ++j) {
    if (fixed_T) { J[S * N + j] = 0.0; continue; }
    double dnum = 0.0, dden = 0.0;
    for (int k = 0; k < S; ++k) {
      dnum += H[k] * dw[k * N + j];
      dden += Cp[k] * dC[k * N + j];
    }
    if (j == S)
      for (int k = 0; k < S; ++k) {
        dnum += Cp[k] * wd[k];                       /* dH_k/dT = Cp_k */
        dden += C[k] * dCp[k];
      }
    J[S * N + j] = -dnum / den + num * dden / (den * den);
  }
  free(C);
  return 0;
}

/* ------------------------------------------------------------ QSS closure -- */

int orc_lu(int n, double *a, int *piv);
void orc_lu_solve(int n, const double *a, const int *piv, double *b);

/* Mixture of the transported species only (the QSS species carry no mass in
 * the state): W_bar, rho and their concentrations into C[species]. */
static void orc_mixture_T(const orc_mech *m, double T, const double *y, double p, double *rho, double *Wbar,
                          double *C) {
  double inv = 0.0;
  for (int i = 0; i < m->ST; ++i) inv += y[i] / m->W[m->tsp[i]];
  double Wb = 1.0 / inv;
  double r = (p * 10.0) * Wb / (ORC_RU * 1.0e7 * T);
  for (int k = 0; k < m->S; ++k) C[k] = 0.0;
  for (int i = 0; i < m->ST; ++i) C[m->tsp[i]] = r * y[i] / m->W[m->tsp[i]];
  *rho = r;
  *Wbar = Wb;
}

/* Concentrations of the QSS species from the algebraic closure (Eq. 4-6):
 * with the quadratic couplings removed, every kept direction holds at most
 * one QSS concentration as a factor, so the QSS production rates are affine,
 *   wdot_QSS = A C_QSS - b,
 * with A_mn = sum_j nu_mj (d'_nj q_fj - d''_nj q_bj)/C_n (n a reactant of the
 * forward / a product of the reverse direction) and b the negated part free
 * of QSS concentrations.  A C_QSS = b is solved as one dense system with
 * partial pivoting: the plain definition of the result the paper reaches by
 * solving the strongly connected groups in dependency order (App. B).
 * C holds the transported concentrations; the QSS entries are filled in.
 * K[j] receives the rate constants.  Returns 0, or 1 if A is singular. */
static int orc_qss_solve(const orc_mech *m, double T, double *C, const double *G, const double *H, double Mconc,
                         orc_k *K) {
  const int nq = m->nq, R = m->R;
  double *A = calloc((size_t)nq * nq + nq, sizeof(double)), *b = A + nq * nq;
  int *piv = malloc(sizeof(int) * nq);
  for (int j = 0; j < R; ++j) {
    const orc_reaction *x = &m->rx[j];
    double Mj = orc_third_body(m, j, C, Mconc);
    K[j] = orc_rate_constants(m, j, T, G, H, Mj);
    double mfac = (x->type == 1) ? Mj : 1.0;
    int any = 0;
    for (int q = 0; q < nq; ++q) any |= m->nu[m->qsp[q] * R + j] != 0;
    if (!any) continue;
    /* forward: k_f times the reactant concentrations, one of which may be QSS */
    if (!x->drop_f) {
      double c = mfac * K[j].kf;
      int n = -1;
      for (int i = 0; i < x->nr; ++i) {
        if (m->isq[x->r[i]] >= 0) n = m->isq[x->r[i]];
        else c *= C[x->r[i]];
      }
      for (int q = 0; q < nq; ++q) {
        int nu = m->nu[m->qsp[q] * R + j];
        if (!nu) continue;
        if (n >= 0) A[q * nq + n] += nu * c;
        else b[q] -= nu * c;
      }
    }
    if (x->rev && !x->drop_r) {
      double c = mfac * K[j].kr;
      int n = -1;
      for (int i = 0; i < x->np; ++i) {
        if (m->isq[x->p[i]] >= 0) n = m->isq[x->p[i]];
        else c *= C[x->p[i]];
      }
      for (int q = 0; q < nq; ++q) {
        int nu = m->nu[m->qsp[q] * R + j];
        if (!nu) continue;
        if (n >= 0) A[q * nq + n] -= nu * c;
        else b[q] += nu * c;
      }
    }
  }
  int info = orc_lu(nq, A, piv);
  if (!info) orc_lu_solve(nq, A, piv, b);
  for (int q = 0; q < nq; ++q) C[m->qsp[q]] = info ? NAN : b[q];
  free(A);
  free(piv);
  return info != 0;
}

/* Net production rates of every species at concentrations C (QSS ones
 * included) with the linearised directions removed. */
static void orc_qss_wdot(const orc_mech *m, const double *C, double Mconc, const orc_k *K, double *wdot) {
  const int S = m->S, R = m->R;
  for (int k = 0; k < S; ++k) wdot[k] = 0.0;
  for (int j = 0; j < R; ++j) {
    const orc_reaction *x = &m->rx[j];
    double Mj = orc_third_body(m, j, C, Mconc);
    double qf = 0.0, qr = 0.0;
    if (!x->drop_f) {
      qf = K[j].kf;
      for (int i = 0; i < x->nr; ++i) qf *= C[x->r[i]];
    }
    if (x->rev && !x->drop_r) {
      qr = K[j].kr;
      for (int i = 0; i < x->np; ++i) qr *= C[x->p[i]];
    }
    double q = qf - qr;
    if (x->type == 1) q *= Mj;
    for (int k = 0; k < S; ++k) wdot[k] += m->nu[k * R + j] * q;
  }
}

/* QSS concentrations (mol/cm^3) and the production rates of the transported
 * species at a state (T, Y of the transported species), for tests. */
int orc_qss_rates(const orc_mech *m, double T, const double *Y, double p, double *Cq, double *wdot_T) {
  const int S = m->S;
  double *C = malloc(sizeof(double) * 5 * S), *H = C + S, *G = H + S, *Sm = G + S, *wd = Sm + S;
  orc_k *K = malloc(sizeof(orc_k) * (m->R > 0 ? m->R : 1));
  double rho, Wbar;
  orc_mixture_T(m, T, Y, p, &rho, &Wbar, C);
  orc_thermo(m, T, H, Sm, NULL, G);
  for (int k = 0; k < S; ++k) G[k] /= ORC_RU * T;
  double Mconc = 0.0;
  for (int i = 0; i < m->ST; ++i) Mconc += C[m->tsp[i]];
  int bad = orc_qss_solve(m, T, C, G, H, Mconc, K);
  orc_qss_wdot(m, C, Mconc, K, wd);
  if (Cq) for (int q = 0; q < m->nq; ++q) Cq[q] = C[m->qsp[q]];
  if (wdot_T) for (int i = 0; i < m->ST; ++i) wdot_T[i] = wd[m->tsp[i]];
  free(C);
  free(K);
  return bad;
}

/* Reduced right-hand side, y = (Y of the transported species, T). */
static int orc_rhs_qss(const orc_mech *m, const double *y, double p, int fixed_T, double *f) {
  const int S = m->S, ST = m->ST;
  double T = y[ST];
  double *C = malloc(sizeof(double) * 6 * S), *H = C + S, *G = H + S, *Sm = G + S, *Cp = Sm + S, *wd = Cp + S;
  orc_k *K = malloc(sizeof(orc_k) * (m->R > 0 ? m->R : 1));
  double rho, Wbar;
  orc_mixture_T(m, T, y, p, &rho, &Wbar, C);
  orc_thermo(m, T, H, Sm, Cp, G);
  for (int k = 0; k < S; ++k) G[k] /= ORC_RU * T;
  double Mconc = 0.0;
  for (int i = 0; i < ST; ++i) Mconc += C[m->tsp[i]];
  orc_qss_solve(m, T, C, G, H, Mconc, K);
  orc_qss_wdot(m, C, Mconc, K, wd);
  double num = 0.0, den = 0.0;
  for (int i = 0; i < ST; ++i) {
    int k = m->tsp[i];
    f[i] = m->W[k] * wd[k] / rho;
    num += H[k] * wd[k];
    den += C[k] * Cp[k];
  }
  f[ST] = fixed_T ? 0.0 : -num / den;
  free(C);
  free(K);
  return 0;
}

/* Jacobian of the reduced right-hand side (the paper's QSS chain rule,
 * Sec. 3.2): the QSS concentrations depend on the transported ones and on T
 * through the closure wdot_QSS = 0, so with the concentration-space blocks
 * A_TT, A_TQ, A_QT, A_QQ of d wdot/dC (the linearised mechanism, at the
 * closure's C) and the T-derivatives b_T, b_Q at fixed C,
 *   d wdot_T/dC_T = A_TT - A_TQ A_QQ^-1 A_QT,  d wdot_T/dT = b_T - A_TQ A_QQ^-1 b_Q
 * (A_QQ is the closure matrix).  The chain rule through C(Y, T) and rho(Y, T)
 * of the transported mixture then follows as in orc_jac. */
static int orc_jac_qss(const orc_mech *m, const double *y, double p, int fixed_T, double *J) {
  const int S = m->S, R = m->R, ST = m->ST, nq = m->nq, N = ST + 1;
  double T = y[ST];
  double *C = malloc(sizeof(double) * (size_t)(8 * S + S * S + nq * (ST + 1) + nq * nq + 2 * ST * N + N));
  double *H = C + S, *Cp = H + S, *G = Cp + S, *Sm = G + S, *wd = Sm + S, *b = wd + S, *dCp = b + S;
  double *A = dCp + S;              /* [S][S] d wdot_k / dC_c over all species */
  double *X = A + S * S;            /* [nq][ST+1]: A_QQ^-1 [A_QT | b_Q] */
  double *Aqq = X + nq * (ST + 1);  /* [nq][nq] */
  double *dC = Aqq + nq * nq;       /* [ST][N] */
  double *dw = dC + ST * N;         /* [ST][N] */
  double *drho = dw + ST * N;       /* [N] */
  orc_k *K = malloc(sizeof(orc_k) * (R > 0 ? R : 1));
  int *piv = malloc(sizeof(int) * (nq > 0 ? nq : 1));
  double rho, Wbar;
  orc_mixture_T(m, T, y, p, &rho, &Wbar, C);
  orc_thermo(m, T, H, Sm, Cp, G);
  orc_dcp_dT(m, T, dCp);
  for (int k = 0; k < S; ++k) G[k] /= ORC_RU * T;
  double Mconc = 0.0;
  for (int i = 0; i < ST; ++i) Mconc += C[m->tsp[i]];
  orc_qss_solve(m, T, C, G, H, Mconc, K);
  orc_qss_wdot(m, C, Mconc, K, wd);
  for (int i = 0; i < S * S; ++i) A[i] = 0.0;
  for (int k = 0; k < S; ++k) b[k] = 0.0;
  for (int j = 0; j < R; ++j) {
    const orc_reaction *x = &m->rx[j];
    double Mj = orc_third_body(m, j, C, Mconc);
    double kf = x->drop_f ? 0.0 : K[j].kf, dkf = x->drop_f ? 0.0 : K[j].dkf;
    double dkf_dM = x->drop_f ? 0.0 : K[j].dkf_dM;
    int rev = x->rev && !x->drop_r;
    double kr = rev ? K[j].kr : 0.0, dkr = rev ? K[j].dkr : 0.0, dkr_dM = rev ? K[j].dkr_dM : 0.0;
    double pf = 1.0, pr = 1.0;
    for (int i = 0; i < x->nr; ++i) pf *= C[x->r[i]];
    for (int i = 0; i < x->np; ++i) pr *= C[x->p[i]];
    double mfac = (x->type == 1) ? Mj : 1.0;
    double dq_dT = mfac * (dkf * pf - dkr * pr);
    for (int c = 0; c < S; ++c) {
      double dpf = 0.0, dpr = 0.0;
      for (int i = 0; i < x->nr; ++i) {
        if (x->r[i] != c) continue;
        double t = 1.0;
        for (int i2 = 0; i2 < x->nr; ++i2) if (i2 != i) t *= C[x->r[i2]];
        dpf += t;
      }
      for (int i = 0; i < x->np; ++i) {
        if (x->p[i] != c) continue;
        double t = 1.0;
        for (int i2 = 0; i2 < x->np; ++i2) if (i2 != i) t *= C[x->p[i2]];
        dpr += t;
      }
      double dq = mfac * (kf * dpf - kr * dpr);
      double eps = (x->type == 0) ? 0.0 : orc_efficiency(m, x, c);
      if (x->type == 1) dq += eps * (kf * pf - kr * pr);
      if (x->type == 2) dq += eps * (dkf_dM * pf - dkr_dM * pr);
      for (int k = 0; k < S; ++k) A[k * S + c] += m->nu[k * R + j] * dq;
    }
    for (int k = 0; k < S; ++k) b[k] += m->nu[k * R + j] * dq_dT;
  }
  /* X = A_QQ^-1 [A_QT | b_Q] */
  for (int q = 0; q < nq; ++q) {
    for (int q2 = 0; q2 < nq; ++q2) Aqq[q * nq + q2] = A[m->qsp[q] * S + m->qsp[q2]];
  }
  orc_lu(nq, Aqq, piv);
  double *col = malloc(sizeof(double) * (nq > 0 ? nq : 1));
  for (int c = 0; c <= ST; ++c) {
    for (int q = 0; q < nq; ++q) col[q] = c < ST ? A[m->qsp[q] * S + m->tsp[c]] : b[m->qsp[q]];
    orc_lu_solve(nq, Aqq, piv, col);
    for (int q = 0; q < nq; ++q) X[q * (ST + 1) + c] = col[q];
  }
  free(col);
  /* dC_m/dY_j = delta_mj rho/W_m - C_m Wbar/W_j ; dC_m/dT = -C_m/T (transported) */
  for (int a = 0; a < ST; ++a) {
    int ka = m->tsp[a];
    for (int j = 0; j < ST; ++j) dC[a * N + j] = (a == j ? rho / m->W[ka] : 0.0) - C[ka] * Wbar / m->W[m->tsp[j]];
    dC[a * N + ST] = -C[ka] / T;
  }
  for (int j = 0; j < ST; ++j) drho[j] = -rho * Wbar / m->W[m->tsp[j]];
  drho[ST] = -rho / T;
  /* reduced concentration-space Jacobian, then the chain rule */
  for (int a = 0; a < ST; ++a) {
    int ka = m->tsp[a];
    for (int j = 0; j < N; ++j) {
      double s = 0.0;
      for (int c = 0; c < ST; ++c) {
        double ared = A[ka * S + m->tsp[c]];
        for (int q = 0; q < nq; ++q) ared -= A[ka * S + m->qsp[q]] * X[q * (ST + 1) + c];
        s += ared * dC[c * N + j];
      }
      if (j == ST) {
        double bred = b[ka];
        for (int q = 0; q < nq; ++q) bred -= A[ka * S + m->qsp[q]] * X[q * (ST + 1) + ST];
        s += bred;
      }
      dw[a * N + j] = s;
    }
  }
  for (int a = 0; a < ST; ++a) {
    int ka = m->tsp[a];
    for (int j = 0; j < N; ++j)
      J[a * N + j] = m->W[ka] / rho * dw[a * N + j] - m->W[ka] * wd[ka] / (rho * rho) * drho[j];
  }
  double num = 0.0, den = 0.0;
  for (int a = 0; a < ST; ++a) {
    int ka = m->tsp[a];
    num += H[ka] * wd[ka];
    den += C[ka] * Cp[ka];
  }
  for (int j = 0; j < N; ++j) {
    if (fixed_T) { J[ST * N + j] = 0.0; continue; }
    double dnum = 0.0, dden = 0.0;
    for (int a = 0; a < ST; ++a) {
      int ka = m->tsp[a];
      dnum += H[ka] * dw[a * N + j];
      dden += Cp[ka] * dC[a * N + j];
    }
    if (j == ST)
      for (int a = 0; a < ST; ++a) {
        int ka = m->tsp[a];
        dnum += Cp[ka] * wd[ka];
        dden += C[ka] * dCp[ka];
      }
    J[ST * N + j] = -dnum / den + num * dden / (den * den);
  }
  free(C);
  free(K);
  free(piv);
  return 0;
}

/* ------------------------------------------------------------ linear algebra */

/* In-place LU with partial pivoting (row swaps; the first row index wins among
 * equal magnitudes).  Returns 0, or j+1 if column j has no nonzero pivot. */
int orc_lu(int n, double *a, int *piv) {
  int info = 0;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = fabs(a[k * n + k]);
    for (int i = k + 1; i < n; ++i)
      if (fabs(a[i * n + k]) > best) { best = fabs(a[i * n + k]); p = i; }
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) { double t = a[k * n + j]; a[k * n + j] = a[p * n + j]; a[p * n + j] = t; }
    if (a[k * n + k] == 0.0) { if (!info) info = k + 1; continue; }
    for (int i = k + 1; i < n; ++i) {
      double l = a[i * n + k] / a[k * n + k];
      a[i * n + k] = l;
      for (int j = k + 1; j < n; ++j) a[i * n + j] -= l * a[k * n + j];
    }
  }
  return info;
}

/* Solve A x = b with the factors of orc_lu; b is overwritten by x. */
void orc_lu_solve(int n, const double *a, const int *piv, double *b) {
  for (int k = 0; k < n; ++k)
    if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) b[i] -= a[i * n + j] * b[j];
  for (int i = n - 1; i >= 0; --i) {
    for (int j = i + 1; j < n; ++j) b[i] -= a[i * n + j] * b[j];
    b[i] /= a[i * n + i];
  }
}

/* ------------------------------------------------------- enthalpy inversion */

/* Mixture specific enthalpy h = sum_k Y_k H_k(T)/W_k (J/g). */
double orc_enthalpy(const orc_mech *m, double T, const double *Y) {
  double h = 0.0;
  double *H = malloc(sizeof(double) * m->S);
  orc_thermo(m, T, H, NULL, NULL, NULL);
  for (int i = 0; i < m->ST; ++i) h += Y[i] * H[m->tsp[i]] / m->W[m->tsp[i]];
  free(H);
  return h;
}

/* Temperature with mixture enthalpy h at composition Y.  With linear cp the
 * mixture enthalpy is alpha + beta T + gamma T^2; the positive root is taken in
 * the cancellation-free form T = 2c / (beta + sqrt(beta^2 + 4 gamma c)),
 * c = h - alpha. */
double orc_temperature_from_h(const orc_mech *m, double h, const double *Y) {
  int any_nasa = 0;
  for (int k = 0; k < m->S; ++k) any_nasa |= m->nasa[k];
  if (any_nasa) {
    /* Newton on h(T) = h with dh/dT = cp > 0, kept inside a shrinking bracket */
    double lo = 10.0, hi = 10000.0, T = 1000.0;
    double *H = malloc(sizeof(double) * 2 * m->S), *Cp = H + m->S;
    for (int it = 0; it < 200; ++it) {
      orc_thermo(m, T, H, NULL, Cp, NULL);
      double g = -h, dg = 0.0;
      for (int i = 0; i < m->ST; ++i) {
        int k = m->tsp[i];
        g += Y[i] * H[k] / m->W[k];
        dg += Y[i] * Cp[k] / m->W[k];
      }
      if (g > 0) hi = T; else lo = T;
      double Tn = T - g / dg;
      if (!(Tn > lo && Tn < hi)) Tn = 0.5 * (lo + hi);
      if (fabs(Tn - T) <= 1e-13 * T) { T = Tn; break; }
      T = Tn;
    }
    free(H);
    return T;
  }
  double al = 0.0, be = 0.0, ga = 0.0;
  for (int i = 0; i < m->ST; ++i) {
    int k = m->tsp[i];
    double w = Y[i] / m->W[k];
    al += w * (m->hf[k] - ORC_RU * m->a0[k] * ORC_TREF - ORC_RU * m->a1[k] * ORC_TREF * ORC_TREF / 2.0);
    be += w * ORC_RU * m->a0[k];
    ga += w * ORC_RU * m->a1[k] / 2.0;
  }
  double c = h - al;
  return 2.0 * c / (be + sqrt(be * be + 4.0 * ga * c));
}

/* ------------------------------------------------------------- integrator -- */

typedef struct {
  int max_steps;       /* attempts per cell before the cell is declared failed */
  int q_max;           /* highest BDF order, 1..5 */
  int fixed_T;         /* hold T constant: f_T = 0, no projection */
  int fixed_step_n;    /* >0: n equal steps, order ramps 1..q_max, no error test, Newton to 1e-10 */
  int jac_mode;        /* Newton Jacobian: 0 analytic (Eq. 7), 1 difference quotients in every
                          column, 2 analytic species columns with a difference-quotient T column */
  int jac_reuse;       /* 1: keep the factored Newton matrix across attempts while it is recent
                          (see orc_integrate_cell); 0 (the default reading): a fresh Jacobian and
                          LU every attempt */
} orc_opts;

typedef struct {
  int status;          /* 0 ok, 1 max_steps, 2 step size underflow, 3 bad input */
  int steps, attempts, n_rhs, n_jac, n_newton, n_etf, n_nnf;
  int n_clip;          /* mass fractions set to zero by the positivity projection */
  double clip_mass;    /* their total magnitude (the mass the projection added) */
} orc_cell_stats;

#define ORC_QMAX 5

/* WRMS norm over all N components with weights w: sqrt(sum (v_i w_i)^2 / n).
 * Cold cells can have right-hand sides near 1e240, whose squares overflow;
 * when the plain sum is not finite the same norm is taken as
 * M sqrt(sum (v_i w_i / M)^2 / n) with M = max |v_i w_i|. */
static double orc_wrms(int n, const double *v, const double *w) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += (v[i] * w[i]) * (v[i] * w[i]);
  if (isfinite(s)) return sqrt(s / n);
  double M = 0.0;
  for (int i = 0; i < n; ++i)
    if (fabs(v[i] * w[i]) > M) M = fabs(v[i] * w[i]);
  if (!isfinite(M)) return M;
  s = 0.0;
  for (int i = 0; i < n; ++i) s += (v[i] * w[i] / M) * (v[i] * w[i] / M);
  return M * sqrt(s / n);
}

/* Change the step size by the ratio r: the backward differences D_1..D_m of
 * the interpolating polynomial are mapped to the new spacing by D <- D (R U)
 * with R_ij = prod_{l=1..i} (l - 1 - j r)/l and U = R at r = 1 (Shampine &
 * Reichelt's quasi-constant-step BDF).  D[j] points at the j-th difference. */
static void orc_rescale(int n, double **D, int mdim, double r) {
  double Rm[ORC_QMAX + 1][ORC_QMAX + 1], Um[ORC_QMAX + 1][ORC_QMAX + 1], RU[ORC_QMAX + 1][ORC_QMAX + 1];
  double tmp[ORC_QMAX + 1];
  for (int j = 1; j <= mdim; ++j) {
    double pr = 1.0, pu = 1.0;
    for (int i = 1; i <= mdim; ++i) {
      pr *= (i - 1 - j * r) / i;
      pu *= (double)(i - 1 - j) / i;
      Rm[i][j] = pr;
      Um[i][j] = pu;
    }
  }
  for (int i = 1; i <= mdim; ++i)
    for (int j = 1; j <= mdim; ++j) {
      double s = 0.0;
      for (int l = 1; l <= mdim; ++l) s += Rm[i][l] * Um[l][j];
      RU[i][j] = s;
    }
  for (int c = 0; c < n; ++c) {
    for (int j = 1; j <= mdim; ++j) {
      double s = 0.0;
      for (int i = 1; i <= mdim; ++i) s += D[i][c] * RU[i][j];
      tmp[j] = s;
    }
    for (int j = 1; j <= mdim; ++j) D[j][c] = tmp[j];
  }
}

/* Integrate one cell over [0, dt].  y holds (Y_1..Y_S, T) and is overwritten
 * with the state at dt (or at the last accepted time if the cell fails).
 *
 * Variable-order (1..q_max) BDF in backward differences: D_0 = y_n and D_j the
 * j-th backward difference.  For order k the predictor is y0 = sum_{j<=k} D_j
 * and the corrector d = y_{n+1} - y0 solves
 *     d - (h/g_k) f(y0 + d) + psi = 0,   psi = (1/g_k) sum_{j=1..k} g_j D_j,
 * g_j = sum_{i<=j} 1/i.  Newton uses M = I - (h/g_k) J(y0) with J and the LU
 * of M fresh every attempt; it has converged when ||delta|| <= 0.03 and has
 * failed when ||delta_m|| > 2 ||delta_{m-1}|| or after 4 iterations (h /= 4).
 * The local error estimate ||d||/(k+1) <= 1 accepts the step (norm: WRMS with
 * weights 1/(rtol |y_n| + atol)).  The step size and order are held until
 * k+2 steps have been accepted with them (quasi-constant step size); then the
 * error estimates for orders k-1 (||D_k||/k), k (||d||/(k+1)) and k+1
 * (||d - D_{k+1}||/(k+2)) give step factors 1/(1.3 e^(1/k)), 1/(1.2 e^(1/(k+1)))
 * and 1/(1.4 e^(1/(k+2))); the largest wins if it exceeds 1 (capped at 10).
 * An error test failure shrinks h by max(0.2, 0.9 e^(-1/(k+1))); three in a
 * row drop to order 1 with h /= 10.  When t + 1.1 h reaches dt the step is set
 * to end exactly at dt.  Every change of h rescales the
 * differences D_1..D_{min(k+1,q_max)}.  A converged corrector that leaves a
 * mass fraction below -atol is rejected like a failed error test (h /= 4; an
 * inequality constraint Y >= -atol in CVODE's manner): the higher BDF orders
 * can extrapolate a decaying species below zero, and accepting that sets up
 * a cycle of overshoot and Newton failure at the scale of atol.  After every
 * accepted step a mass fraction still below zero is set to zero together
 * with all of its backward differences (projection onto Y >= 0, Sandu 2001:
 * with reverse rate constants as large as these, a species left below zero
 * drives reactions that share it on both sides backwards and the solution
 * runs away; the reset differences make the next predictor hold it at zero).  T is integrated
 * through its own equation and is not projected: moving T after a step moves
 * the fast partial equilibria with it, and the next step then sees a jump no
 * step size above the round-off floor can resolve.  The mixture enthalpy is
 * therefore conserved to the integration tolerance. */
/* Columns j0..N-1 of J = df/dy by one-sided difference quotients at y, the
 * finite-difference Jacobian the paper compares its analytic one against
 * (Sec. 3.2; its T column is taken this way in Sec. 3.2.2).  The increment
 * is the dense difference-quotient rule of the SUNDIALS CVODE documentation:
 *   inc_j = max(sqrt(u) |y_j|, m / w_j),  m = 1000 |h| u N ||f(y)||_w  (1 if that norm is 0),
 * with u the unit roundoff, w the error weights and h the current step.
 * fy = f(y) is given; each column costs one right-hand side.  Returns the
 * number of right-hand sides evaluated. */
static int orc_jac_dq(const orc_mech *m, const double *y, double p, int fixed_T, const double *fy,
                      const double *w, double h, int j0, double *J, double *ytmp, double *f1) {
  const int N = m->ST + 1;
  const double u = 2.220446049250313e-16;
  const double fnorm = orc_wrms(N, fy, w);
  const double minc = fnorm != 0.0 ? 1000.0 * fabs(h) * u * N * fnorm : 1.0;
  for (int j = j0; j < N; ++j) {
    double a = sqrt(u) * fabs(y[j]), b = minc / w[j];
    double inc = a > b ? a : b;
    for (int i = 0; i < N; ++i) ytmp[i] = y[i];
    ytmp[j] = y[j] + inc;
    orc_rhs(m, ytmp, p, fixed_T, f1);
    for (int i = 0; i < N; ++i) J[i * N + j] = (f1[i] - fy[i]) / inc;
  }
  return N - j0;
}

/* The difference-quotient Jacobian at one state (all columns), for tests. */
int orc_jac_fd(const orc_mech *m, const double *y, double p, int fixed_T, const double *w, double h, double *J) {
  const int N = m->ST + 1;
  double *t = malloc(sizeof(double) * 3 * (size_t)N);
  orc_rhs(m, y, p, fixed_T, t);
  int nr = orc_jac_dq(m, y, p, fixed_T, t, w, h, 0, J, t + N, t + 2 * N);
  free(t);
  return nr;
}

static void orc_integrate_cell(const orc_mech *m, double *y, double p, double dt, double rtol, double atol,
                               const orc_opts *o, orc_cell_stats *st) {
  int S = m->ST, N = S + 1;   /* state: the transported species and T */
  int q_max = o->q_max < 1 ? 1 : (o->q_max > ORC_QMAX ? ORC_QMAX : o->q_max);
  double *buf = malloc(sizeof(double) * (size_t)(N * (ORC_QMAX + 3 + 10) + N * N));
  double *D[ORC_QMAX + 3];
  for (int j = 0; j < ORC_QMAX + 3; ++j) D[j] = buf + j * N;
  double *w = buf + (ORC_QMAX + 3) * N, *pred = w + N, *psi = pred + N, *d = psi + N, *f = d + N;
  double *ytmp = f + N, *rhs = ytmp + N, *e = rhs + N, *fq = e + N, *yq = fq + N, *Mx = yq + N;
  int *piv = malloc(sizeof(int) * N);
  memset(st, 0, sizeof *st);
  double g[ORC_QMAX + 2];
  g[0] = 0.0;
  for (int j = 1; j <= ORC_QMAX + 1; ++j) g[j] = g[j - 1] + 1.0 / j;
  int fixedT = o->fixed_T;
  int fixed = o->fixed_step_n > 0;
  double T0 = y[S];
  if (!(T0 > 0.0) || !isfinite(T0) || !(dt > 0.0)) { st->status = 3; goto out; }
  for (int k = 0; k < S; ++k) if (!isfinite(y[k])) { st->status = 3; goto out; }
  for (int j = 0; j < ORC_QMAX + 3; ++j) for (int i = 0; i < N; ++i) D[j][i] = 0.0;
  for (int i = 0; i < N; ++i) D[0][i] = y[i];
  orc_rhs(m, D[0], p, fixedT, f);
  st->n_rhs++;
  for (int i = 0; i < N; ++i) w[i] = 1.0 / (rtol * fabs(D[0][i]) + atol);
  double h;
  if (fixed) {
    h = dt / o->fixed_step_n;
  } else {
    double nf = orc_wrms(N, f, w);
    h = dt;
    if (nf * dt > 1.0) h = 1.0 / nf;
  }
  for (int i = 0; i < N; ++i) D[1][i] = h * f[i];
  int k = 1, etf = 0, nk = 0;   /* nk: accepted steps since the last change of h or order */
  int have_lu = 0, steps_lu = 0, stale_fail = 0;   /* state of the factored Newton matrix */
  double c_lu = 0.0;
  double t = 0.0;
  while (t < dt) {
    if (st->attempts >= o->max_steps) { st->status = 1; break; }
    st->attempts++;
    int last = 0;
    if (fixed) {
      last = (st->steps + 1 == o->fixed_step_n);
    } else if (t + 1.1 * h >= dt) {
      /* end exactly at dt: stretch the step by up to 10% or shorten it, so
       * that no sliver below the resolution of t is left over */
      double hn = dt - t;
      orc_rescale(N, D, k + 1 <= q_max ? k + 1 : q_max, hn / h);
      h = hn;
      nk = 0;
      last = 1;
    }
    /* no progress possible: h below 16 ulp of t (or underflowing at t = 0) */
    if (!(h > 16.0 * 2.220446049250313e-16 * t) || !(h >= 1e-290)) { st->status = 2; break; }
    for (int i = 0; i < N; ++i) w[i] = 1.0 / (rtol * fabs(D[0][i]) + atol);
    for (int i = 0; i < N; ++i) {
      double sp = D[0][i], ss = 0.0;
      for (int j = 1; j <= k; ++j) { sp += D[j][i]; ss += g[j] * D[j][i]; }
      pred[i] = sp;
      psi[i] = ss / g[k];
    }
    double c = h / g[k];
    /* Newton matrix M = I - c J, factored.  With reuse (CVODE's policy for
     * its Newton matrix, Sec. 3.2) the factors of an earlier attempt are kept
     * while they are recent: c within 30% of the c they were formed with,
     * fewer than 20 accepted steps since, and no Newton failure with them
     * (a failure retries the same step with a fresh matrix).  Otherwise the
     * Jacobian is evaluated at the predictor and M factored afresh. */
    int fresh = !o->jac_reuse || !have_lu || fabs(c / c_lu - 1.0) > 0.3 || st->steps - steps_lu >= 20 ||
                stale_fail;
    if (fresh) {
      if (o->jac_mode == 1) {
        orc_rhs(m, pred, p, fixedT, fq);   /* f(pred): the first Newton residual evaluates it again */
        st->n_rhs += orc_jac_dq(m, pred, p, fixedT, fq, w, h, 0, Mx, yq, e);
      } else {
        orc_jac(m, pred, p, fixedT, Mx);
        if (o->jac_mode == 2) {
          orc_rhs(m, pred, p, fixedT, fq);
          st->n_rhs += orc_jac_dq(m, pred, p, fixedT, fq, w, h, S, Mx, yq, e);
        }
      }
      st->n_jac++;
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) Mx[i * N + j] = (i == j ? 1.0 : 0.0) - c * Mx[i * N + j];
      orc_lu(N, Mx, piv);
      have_lu = 1;
      c_lu = c;
      steps_lu = st->steps;
      stale_fail = 0;
    }
    for (int i = 0; i < N; ++i) d[i] = 0.0;
    int conv = 0;
    double prev = 0.0;
    int maxit = fixed ? 50 : 4;
    double ntol = fixed ? 1e-10 : 0.03;
    for (int it = 1; it <= maxit; ++it) {
      for (int i = 0; i < N; ++i) ytmp[i] = pred[i] + d[i];
      orc_rhs(m, ytmp, p, fixedT, f);
      st->n_rhs++;
      st->n_newton++;
      for (int i = 0; i < N; ++i) rhs[i] = -(d[i] - c * f[i] + psi[i]);
      orc_lu_solve(N, Mx, piv, rhs);
      for (int i = 0; i < N; ++i) d[i] += rhs[i];
      double nrm = orc_wrms(N, rhs, w);
      if (nrm <= ntol) { conv = 1; break; }
      if (it > 1 && nrm > 2.0 * prev) break;
      prev = nrm;
    }
    if (!conv && !fixed && !fresh) {   /* a kept matrix failed: same step, fresh matrix */
      st->n_nnf++;
      stale_fail = 1;
      continue;
    }
    if (!conv && !fixed) {
      st->n_nnf++;
      orc_rescale(N, D, k + 1 <= q_max ? k + 1 : q_max, 0.25);
      h *= 0.25;
      nk = 0;
      continue;
    }
    /* inequality constraint: a corrector with a mass fraction below -atol is
     * rejected like a failed error test (h /= 4) */
    if (!fixed) {
      int viol = 0;
      for (int i = 0; i < S; ++i)
        if (pred[i] + d[i] < -atol) viol = 1;
      if (viol) {
        st->n_etf++;
        orc_rescale(N, D, k + 1 <= q_max ? k + 1 : q_max, 0.25);
        h *= 0.25;
        nk = 0;
        continue;
      }
    }
    double err = orc_wrms(N, d, w) / (k + 1);
    if (!fixed && !(err <= 1.0)) {
      st->n_etf++;
      etf++;
      double r;
      if (etf >= 3) {
        k = 1;
        nk = 0;
        r = 0.1;
      } else {
        r = 0.9 * pow(err, -1.0 / (k + 1));
        if (r < 0.2) r = 0.2;
      }
      orc_rescale(N, D, k + 1 <= q_max ? k + 1 : q_max, r);
      h *= r;
      nk = 0;
      continue;
    }
    /* accept: D_{k+2} = d - D_{k+1}, D_{k+1} = d, then D_j += D_{j+1}, j = k..0 */
    if (k < q_max)
      for (int i = 0; i < N; ++i) D[k + 2][i] = d[i] - D[k + 1][i];
    for (int i = 0; i < N; ++i) D[k + 1][i] = d[i];
    for (int j = k; j >= 0; --j)
      for (int i = 0; i < N; ++i) D[j][i] += D[j + 1][i];
    for (int i = 0; i < S; ++i)
      if (D[0][i] < 0.0) {
        st->n_clip++;
        st->clip_mass -= D[0][i];
        for (int j = 0; j < ORC_QMAX + 3; ++j) D[j][i] = 0.0;
      }
    t = last ? dt : t + h;
    st->steps++;
    nk++;
    etf = 0;
    int kn = k;
    double r;
    if (fixed) {
      r = 1.0;
      kn = st->steps + 1 < q_max ? st->steps + 1 : q_max;
    } else {
      r = 1.0;
      if (nk >= k + 2) {
        double tk = 1.2 * pow(err, 1.0 / (k + 1));
        r = tk > 0.1 ? 1.0 / tk : 10.0;
        if (k > 1) {
          double ekm1 = orc_wrms(N, D[k], w) / k;
          double tm = 1.3 * pow(ekm1, 1.0 / k);
          double rm = tm > 0.1 ? 1.0 / tm : 10.0;
          if (rm > r) { r = rm; kn = k - 1; }
        }
        if (k < q_max) {
          double ekp1 = orc_wrms(N, D[k + 2], w) / (k + 2);
          double tp = 1.4 * pow(ekp1, 1.0 / (k + 2));
          double rp = tp > 0.1 ? 1.0 / tp : 10.0;
          if (rp > r) { r = rp; kn = k + 1; }
        }
        if (r > 10.0) r = 10.0;
        if (r <= 1.0) { r = 1.0; kn = k; }
      }
    }
    if (kn != k) { k = kn; nk = 0; }
    if (r != 1.0) { orc_rescale(N, D, k + 1 <= q_max ? k + 1 : q_max, r); nk = 0; }
    h *= r;
  }
  for (int i = 0; i < N; ++i) y[i] = D[0][i];
out:
  free(buf);
  free(piv);
}

/* Integrate n cells in place over dt.  T[n]; Y species-major SoA, Y[k*n + i].
 * stats (optional) receives one record per cell.  nthreads <= 0 uses the
 * OpenMP default.  Returns the number of failed cells. */
int64_t orc_integrate(const orc_mech *m, int64_t n, double *T, double *Y, double p, double dt, double rtol,
                      double atol, const orc_opts *o, orc_cell_stats *stats, int nthreads) {
  int S = m->ST;
  int64_t failed = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : failed)
  for (int64_t i = 0; i < n; ++i) {
    double y[1025];
    orc_cell_stats st;
    for (int k = 0; k < S; ++k) y[k] = Y[(int64_t)k * n + i];
    y[S] = T[i];
    orc_integrate_cell(m, y, p, dt, rtol, atol, o, &st);
    if (st.status == 0 || st.status == 1 || st.status == 2) {
      for (int k = 0; k < S; ++k) Y[(int64_t)k * n + i] = y[k];
      T[i] = y[S];
    }
    if (st.status) failed++;
    if (stats) stats[i] = st;
  }
  return failed;
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
