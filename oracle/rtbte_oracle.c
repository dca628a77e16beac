/*
 * FP64 CPU oracle for the collision integrals of the coupled electron-phonon
 * real-time Boltzmann equation (rt-BTE).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or table with the GPU library; the two meet only at the synthetic
 * inputs.
 *
 * It computes, literally and slowly:
 *   I^{e-ph}[f,N]_nk = -(2 pi/hbar)(1/N_q) sum_{m nu q} |g|^2
 *                      [F_em delta(e_nk - hw_nuq - e_mk+q) + F_abs delta(e_nk + hw_nuq - e_mk+q)]
 *   I^{ph-e}[f,N]_nuq = -(4 pi/hbar)(1/N_k) sum_{m n k} |g|^2 F_abs delta(e_nk + hw_nuq - e_mk+q)
 *     (Methods, Eq. (e-ph); occupation factors F_em, F_abs as defined right after it)
 *   I^{ph-ph}[N]_nuq = -(36 pi/hbar)(1/N_q) sum_{nu' nu'' q' q''} |V3|^2
 *                      [G_em delta(-hw + hw' + hw'') + 2 G_abs delta(hw - hw' + hw'')]
 *     (Methods, Eq. (ph-ph); G_em, G_abs as defined right after it)
 * with the Gaussian delta_sigma(E) = exp(-(E/sigma)^2) / (sigma sqrt(pi)) truncated at
 * |E| <= nsigma*sigma, and every channel that touches a phonon with
 * hbar*omega < hw_cut dropped (Methods, grid-size paragraphs: frequency cutoff).
 *
 * Two independent evaluations are provided:
 *   orc_build / orc_rhs      - over the stored channel lists, one Neumaier-
 *                              compensated sum per destination row;
 *   orc_brute_rhs            - direct loops over the full grid in the paper's
 *                              notation, from dense matrix-element tables, with
 *                              no channel lists (tiny grids only).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define HBAR_EV_FS 0.6582119569 /* eV*fs, CODATA 2018 */
#define PI_ 3.14159265358979323846

typedef struct {
  int32_t n_el, n_ph, n_k_total, n_q_total;
  const double *eps, *hw;
  int64_t n_eph;
  const int32_t *eph_row, *eph_partner, *eph_phonon;
  const double *eph_g2;
  int64_t n_pp;
  const int32_t *pp_row, *pp_a, *pp_b;
  const double *pp_v2;
  double sigma_eph, sigma_pp, nsigma, hw_cut;
} orc_problem;

typedef struct {
  int32_t n_el, n_ph;
  /* e-ph entries in input order */
  int64_t n_eph;
  int32_t *er, *es, *ep;      /* electron row r, partner s, phonon p */
  double *w_em, *w_abs;       /* electron-side weights, 0 when not kept */
  double *w_phe;              /* phonon-side weight of the abs process, 0 when not kept */
  int64_t *el_ptr, *el_idx;   /* entries of electron row r: el_idx[el_ptr[r]..el_ptr[r+1]) */
  int64_t *phe_ptr, *phe_idx; /* abs-kept entries with phonon p */
  /* ph-ph entries in input order */
  int64_t n_pp;
  int32_t *pr, *pa, *pb;
  double *v_em, *v_abs;       /* weights (abs includes its factor 2), 0 when not kept */
  int64_t *pp_ptr, *pp_idx;
  int64_t count_e, count_pe, count_pp;  /* stored channels of the three sums */
} orc_lists;

static double gauss_delta(double x, double sigma) {
  double u = x / sigma;
  return exp(-u * u) / (sigma * sqrt(PI_));
}

/* Stable grouping of `n` items by key into CSR (ptr has nkeys+1 entries). */
static int group_by(int64_t n, const int32_t *key, const unsigned char *use, int32_t nkeys,
                    int64_t **ptr_out, int64_t **idx_out) {
  int64_t *ptr = (int64_t *)calloc((size_t)nkeys + 1, sizeof(int64_t));
  if (!ptr) return -2;
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i)
    if (!use || use[i]) { ptr[key[i] + 1]++; ++m; }
  for (int32_t k = 0; k < nkeys; ++k) ptr[k + 1] += ptr[k];
  int64_t *idx = (int64_t *)malloc((size_t)(m ? m : 1) * sizeof(int64_t));
  int64_t *cur = (int64_t *)malloc((size_t)nkeys * sizeof(int64_t) + 8);
  if (!idx || !cur) { free(ptr); free(idx); free(cur); return -2; }
  memcpy(cur, ptr, (size_t)nkeys * sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i)
    if (!use || use[i]) idx[cur[key[i]]++] = i;
  free(cur);
  *ptr_out = ptr;
  *idx_out = idx;
  return 0;
}

void orc_free(orc_lists *L) {
  if (!L) return;
  free(L->er); free(L->es); free(L->ep); free(L->w_em); free(L->w_abs); free(L->w_phe);
  free(L->el_ptr); free(L->el_idx); free(L->phe_ptr); free(L->phe_idx);
  free(L->pr); free(L->pa); free(L->pb); free(L->v_em); free(L->v_abs);
  free(L->pp_ptr); free(L->pp_idx);
  free(L);
}

/* Build the weighted lists.  status: 0 ok, -1 invalid input, -2 out of memory. */
orc_lists *orc_build(const orc_problem *P, int *status) {
  *status = -1;
  if (P->n_el < 0 || P->n_ph < 0 || P->n_eph < 0 || P->n_pp < 0) return NULL;
  if (P->sigma_eph <= 0 || P->sigma_pp <= 0 || P->nsigma <= 0) return NULL;
  if (P->n_k_total <= 0 || P->n_q_total <= 0) return NULL;
  for (int64_t i = 0; i < P->n_eph; ++i) {
    if (P->eph_row[i] < 0 || P->eph_row[i] >= P->n_el) return NULL;
    if (P->eph_partner[i] < 0 || P->eph_partner[i] >= P->n_el) return NULL;
    if (P->eph_phonon[i] < 0 || P->eph_phonon[i] >= P->n_ph) return NULL;
  }
  for (int64_t i = 0; i < P->n_pp; ++i) {
    if (P->pp_row[i] < 0 || P->pp_row[i] >= P->n_ph) return NULL;
    if (P->pp_a[i] < 0 || P->pp_a[i] >= P->n_ph) return NULL;
    if (P->pp_b[i] < 0 || P->pp_b[i] >= P->n_ph) return NULL;
  }
  *status = -2;
  orc_lists *L = (orc_lists *)calloc(1, sizeof(orc_lists));
  if (!L) return NULL;
  L->n_el = P->n_el;
  L->n_ph = P->n_ph;
  const int64_t ne = P->n_eph, np = P->n_pp;
  const size_t ne1 = (size_t)(ne ? ne : 1), np1 = (size_t)(np ? np : 1);
  L->n_eph = ne;
  L->er = (int32_t *)malloc(ne1 * 4); L->es = (int32_t *)malloc(ne1 * 4); L->ep = (int32_t *)malloc(ne1 * 4);
  L->w_em = (double *)malloc(ne1 * 8); L->w_abs = (double *)malloc(ne1 * 8); L->w_phe = (double *)malloc(ne1 * 8);
  L->n_pp = np;
  L->pr = (int32_t *)malloc(np1 * 4); L->pa = (int32_t *)malloc(np1 * 4); L->pb = (int32_t *)malloc(np1 * 4);
  L->v_em = (double *)malloc(np1 * 8); L->v_abs = (double *)malloc(np1 * 8);
  unsigned char *abs_kept = (unsigned char *)malloc(ne1);
  if (!L->er || !L->es || !L->ep || !L->w_em || !L->w_abs || !L->w_phe || !L->pr || !L->pa ||
      !L->pb || !L->v_em || !L->v_abs || !abs_kept) {
    free(abs_kept); orc_free(L); return NULL;
  }
  /* Electron-side and phonon-side weights of every e-ph entry (Eq. (e-ph)). */
  const double pre_el = (2.0 * PI_ / HBAR_EV_FS) / (double)P->n_q_total;
  const double pre_ph = (4.0 * PI_ / HBAR_EV_FS) / (double)P->n_k_total;
  const double cut_e = P->nsigma * P->sigma_eph;
  int64_t ce = 0, cpe = 0;
#pragma omp parallel for reduction(+ : ce, cpe)
  for (int64_t i = 0; i < ne; ++i) {
    int32_t r = P->eph_row[i], s = P->eph_partner[i], p = P->eph_phonon[i];
    double g2 = P->eph_g2[i], w = P->hw[p];
    L->er[i] = r; L->es[i] = s; L->ep[i] = p;
    L->w_em[i] = 0.0; L->w_abs[i] = 0.0; L->w_phe[i] = 0.0; abs_kept[i] = 0;
    if (w < P->hw_cut) continue;
    double x_em = P->eps[r] - w - P->eps[s];
    double x_abs = P->eps[r] + w - P->eps[s];
    if (fabs(x_em) <= cut_e) { L->w_em[i] = pre_el * g2 * gauss_delta(x_em, P->sigma_eph); ++ce; }
    if (fabs(x_abs) <= cut_e) {
      double d = gauss_delta(x_abs, P->sigma_eph);
      L->w_abs[i] = pre_el * g2 * d;
      L->w_phe[i] = pre_ph * g2 * d;
      abs_kept[i] = 1;
      ++ce; ++cpe;
    }
  }
  /* ph-ph weights (Eq. (ph-ph)); the absorption term carries its factor 2. */
  const double pre_pp = (36.0 * PI_ / HBAR_EV_FS) / (double)P->n_q_total;
  const double cut_p = P->nsigma * P->sigma_pp;
  int64_t cpp = 0;
#pragma omp parallel for reduction(+ : cpp)
  for (int64_t i = 0; i < np; ++i) {
    int32_t l = P->pp_row[i], a = P->pp_a[i], b = P->pp_b[i];
    double v2 = P->pp_v2[i];
    double w = P->hw[l], wa = P->hw[a], wb = P->hw[b];
    L->pr[i] = l; L->pa[i] = a; L->pb[i] = b;
    L->v_em[i] = 0.0; L->v_abs[i] = 0.0;
    if (w < P->hw_cut || wa < P->hw_cut || wb < P->hw_cut) continue;
    double x_em = -w + wa + wb;
    double x_abs = w - wa + wb;
    if (fabs(x_em) <= cut_p) { L->v_em[i] = pre_pp * v2 * gauss_delta(x_em, P->sigma_pp); ++cpp; }
    if (fabs(x_abs) <= cut_p) { L->v_abs[i] = 2.0 * pre_pp * v2 * gauss_delta(x_abs, P->sigma_pp); ++cpp; }
  }
  L->count_e = ce; L->count_pe = cpe; L->count_pp = cpp;
  int rc = 0;
  rc |= group_by(ne, L->er, NULL, P->n_el, &L->el_ptr, &L->el_idx);
  rc |= group_by(ne, L->ep, abs_kept, P->n_ph, &L->phe_ptr, &L->phe_idx);
  rc |= group_by(np, L->pr, NULL, P->n_ph, &L->pp_ptr, &L->pp_idx);
  free(abs_kept);
  if (rc) { orc_free(L); return NULL; }
  *status = 0;
  return L;
}

void orc_counts(const orc_lists *L, int64_t out[3]) {
  out[0] = L->count_e; out[1] = L->count_pe; out[2] = L->count_pp;
}

/* Neumaier (improved Kahan-Babuska) compensated accumulation. */
typedef struct { double s, c, mag, absw, umag, sq; } acc_t;
/* x = W * factor; m = |gain| + |loss| of the factor (unweighted). */
static inline void acc_add(acc_t *a, double w, double x, double m) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
  a->absw += fabs(x);
  a->mag += fabs(w) * m;
  a->umag += m;
  a->sq += x * x;
}

/* Occupation factors, evaluated as printed (gain term minus loss term).
 * Each returns the factor and its two terms' magnitude sum. */
static inline double F_em(double fr, double fs, double Np, double *m) {
  double g = fr * (1.0 - fs) * (1.0 + Np), l = (1.0 - fr) * fs * Np;
  *m = fabs(g) + fabs(l);
  return g - l;
}
static inline double F_abs(double fr, double fs, double Np, double *m) {
  double g = fr * (1.0 - fs) * Np, l = (1.0 - fr) * fs * (1.0 + Np);
  *m = fabs(g) + fabs(l);
  return g - l;
}
static inline double G_em(double N, double Na, double Nb, double *m) {
  double g = N * (Na + 1.0) * (Nb + 1.0), l = (N + 1.0) * Na * Nb;
  *m = fabs(g) + fabs(l);
  return g - l;
}
static inline double G_abs(double N, double Na, double Nb, double *m) {
  double g = N * (Na + 1.0) * Nb, l = (N + 1.0) * Na * (Nb + 1.0);
  *m = fabs(g) + fabs(l);
  return g - l;
}

/* One destination row of y' (row < n_el: electron nk; else phonon nuq).
 * parts: 1 = I^{e-ph}, 2 = I^{ph-e}, 4 = I^{ph-ph}. */
static double row_value(const orc_lists *L, const double *y, int64_t row, int parts, double *S,
                        double *A, double *M, double *Q) {
  const double *f = y, *N = y + L->n_el;
  acc_t a = {0, 0, 0, 0, 0, 0};
  double m;
  if (row < L->n_el) {
    if (parts & 1) {
      const int32_t r = (int32_t)row;
      for (int64_t j = L->el_ptr[r]; j < L->el_ptr[r + 1]; ++j) {
        int64_t i = L->el_idx[j];
        double fr = f[r], fs = f[L->es[i]], Np = N[L->ep[i]];
        if (L->w_em[i] != 0.0) { double F = F_em(fr, fs, Np, &m); acc_add(&a, L->w_em[i], L->w_em[i] * F, m); }
        if (L->w_abs[i] != 0.0) { double F = F_abs(fr, fs, Np, &m); acc_add(&a, L->w_abs[i], L->w_abs[i] * F, m); }
      }
    }
  } else {
    const int32_t p = (int32_t)(row - L->n_el);
    if (parts & 2) {
      for (int64_t j = L->phe_ptr[p]; j < L->phe_ptr[p + 1]; ++j) {
        int64_t i = L->phe_idx[j];
        double F = F_abs(f[L->er[i]], f[L->es[i]], N[p], &m);
        acc_add(&a, L->w_phe[i], L->w_phe[i] * F, m);
      }
    }
    if (parts & 4) {
      for (int64_t j = L->pp_ptr[p]; j < L->pp_ptr[p + 1]; ++j) {
        int64_t i = L->pp_idx[j];
        double Na = N[L->pa[i]], Nb = N[L->pb[i]];
        if (L->v_em[i] != 0.0) { double G = G_em(N[p], Na, Nb, &m); acc_add(&a, L->v_em[i], L->v_em[i] * G, m); }
        if (L->v_abs[i] != 0.0) { double G = G_abs(N[p], Na, Nb, &m); acc_add(&a, L->v_abs[i], L->v_abs[i] * G, m); }
      }
    }
  }
  if (S) *S = a.absw;
  if (A) *A = a.mag;
  if (M) *M = a.umag;
  if (Q) *Q = a.sq;
  return -(a.s + a.c);
}

/* Full right-hand side y' = [I^{e-ph}; I^{ph-e} + I^{ph-ph}] (Eq. (erk_rhs)),
 * restricted to the parts in `parts`.  Optional per-row outputs: S = sum |W F|,
 * A = sum |W| (|gain| + |loss|), M = sum (|gain| + |loss|), Q = sum (W F)^2. */
void orc_rhs(const orc_lists *L, const double *y, double *ydot, int parts, double *S, double *A,
             double *M, double *Q) {
  const int64_t ny = (int64_t)L->n_el + L->n_ph;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t row = 0; row < ny; ++row) {
    double s, a, m, q;
    ydot[row] = row_value(L, y, row, parts, &s, &a, &m, &q);
    if (S) S[row] = s;
    if (A) A[row] = a;
    if (M) M[row] = m;
    if (Q) Q[row] = q;
  }
}

/* Linearized (relaxation-time) rates Gamma_i = -d(ydot_i)/d(y_i) with the
 * partner populations held fixed: the sum over row i's channels of W times
 * the derivative of its occupation factor with respect to the row's own
 * population, from the factor definitions after Eq. (e-ph) and Eq. (ph-ph).
 * On channels whose partner is the row's own state (q = 0 self-scattering)
 * this is the standard scattering rate, not the Jacobian diagonal:
 *   dF_em/df_r  = (1-f_s)(1+N_p) + f_s N_p      dF_abs/df_r = (1-f_s) N_p + f_s (1+N_p)
 *   dF_abs/dN_p = f_r (1-f_s) - (1-f_r) f_s      (ph-e rows)
 *   dG_em/dN    = (N_a+1)(N_b+1) - N_a N_b      dG_abs/dN   = (N_a+1) N_b - N_a (N_b+1)
 * Neumaier-compensated sums; at phonons in equilibrium at temperature T the
 * ph-ph part gives the mode-resolved three-phonon scattering rates. */
static double row_rate(const orc_lists *L, const double *y, int64_t row, int parts, double *mag) {
  const double *f = y, *N = y + L->n_el;
  acc_t a = {0, 0, 0, 0, 0, 0};
  if (row < L->n_el) {
    if (parts & 1) {
      const int32_t r = (int32_t)row;
      for (int64_t j = L->el_ptr[r]; j < L->el_ptr[r + 1]; ++j) {
        int64_t i = L->el_idx[j];
        double fs = f[L->es[i]], Np = N[L->ep[i]];
        if (L->w_em[i] != 0.0) {
          double X = (1.0 - fs) * (1.0 + Np), Y = fs * Np;
          acc_add(&a, L->w_em[i], L->w_em[i] * (X + Y), fabs(X) + fabs(Y));
        }
        if (L->w_abs[i] != 0.0) {
          double X = (1.0 - fs) * Np, Y = fs * (1.0 + Np);
          acc_add(&a, L->w_abs[i], L->w_abs[i] * (X + Y), fabs(X) + fabs(Y));
        }
      }
    }
  } else {
    const int32_t p = (int32_t)(row - L->n_el);
    if (parts & 2) {
      for (int64_t j = L->phe_ptr[p]; j < L->phe_ptr[p + 1]; ++j) {
        int64_t i = L->phe_idx[j];
        double fr = f[L->er[i]], fs = f[L->es[i]];
        double X = fr * (1.0 - fs), Y = (1.0 - fr) * fs;
        acc_add(&a, L->w_phe[i], L->w_phe[i] * (X - Y), fabs(X) + fabs(Y));
      }
    }
    if (parts & 4) {
      for (int64_t j = L->pp_ptr[p]; j < L->pp_ptr[p + 1]; ++j) {
        int64_t i = L->pp_idx[j];
        double Na = N[L->pa[i]], Nb = N[L->pb[i]];
        if (L->v_em[i] != 0.0) {
          double X = (Na + 1.0) * (Nb + 1.0), Y = Na * Nb;
          acc_add(&a, L->v_em[i], L->v_em[i] * (X - Y), fabs(X) + fabs(Y));
        }
        if (L->v_abs[i] != 0.0) {
          double X = (Na + 1.0) * Nb, Y = Na * (Nb + 1.0);
          acc_add(&a, L->v_abs[i], L->v_abs[i] * (X - Y), fabs(X) + fabs(Y));
        }
      }
    }
  }
  if (mag) *mag = a.mag;
  return a.s + a.c;
}

/* Rates of every row; optional mag[i] = sum |W| (|X| + |Y|) over the row's
 * channels, with dF/dx = X +- Y (the magnitude the rate is formed from). */
void orc_rates(const orc_lists *L, const double *y, double *out, int parts, double *mag) {
  const int64_t ny = (int64_t)L->n_el + L->n_ph;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t row = 0; row < ny; ++row) out[row] = row_rate(L, y, row, parts, mag ? mag + row : NULL);
}

/* Largest stored channel weight. */
double orc_max_weight(const orc_lists *L) {
  double m = 0.0;
  for (int64_t i = 0; i < L->n_eph; ++i) {
    m = fmax(m, fmax(fabs(L->w_em[i]), fabs(L->w_abs[i])));
    m = fmax(m, fabs(L->w_phe[i]));
  }
  for (int64_t i = 0; i < L->n_pp; ++i) m = fmax(m, fmax(fabs(L->v_em[i]), fabs(L->v_abs[i])));
  return m;
}

/* Selected rows only (sampled parity at full size). */
void orc_rhs_rows(const orc_lists *L, const double *y, const int64_t *rows, int64_t nrows, double *out,
                  int parts, double *S, double *A) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t j = 0; j < nrows; ++j) {
    double s, a;
    out[j] = row_value(L, y, rows[j], parts, &s, &a, NULL, NULL);
    if (S) S[j] = s;
    if (A) A[j] = a;
  }
}

/* ------------------------------------------------------------------ brute force
 * Direct sums over the full grid (dim 2 or 3, L points per axis) in the
 * paper's notation.  el_of_full[k*n_bands + n] maps the grid state (n,k) to
 * its windowed index (or -1: outside the window, not in the dynamics).
 * g2d[((f*n_bands + m)*n_modes + nu)*N + q] holds |g_{mn nu}(k,q)|^2 for
 * f = k*n_bands + n; v2d[((lam*N + q1)*n_modes + n1)*n_modes + n2] holds
 * |V3|^2 for phonons lam = q*n_modes+nu, (n1,q1), (n2, -(q+q1)). */
static int kplusq(int dim, int L, int k, int q) {
  int ck[3], cq[3];
  if (dim == 2) { ck[0] = k / L; ck[1] = k % L; ck[2] = 0; cq[0] = q / L; cq[1] = q % L; cq[2] = 0; }
  else {
    ck[0] = k / (L * L); ck[1] = (k / L) % L; ck[2] = k % L;
    cq[0] = q / (L * L); cq[1] = (q / L) % L; cq[2] = q % L;
  }
  int c[3];
  for (int i = 0; i < 3; ++i) c[i] = (ck[i] + cq[i]) % L;
  return dim == 2 ? c[0] * L + c[1] : (c[0] * L + c[1]) * L + c[2];
}
static int minusq(int dim, int L, int q) {
  int c[3];
  if (dim == 2) { c[0] = q / L; c[1] = q % L; c[2] = 0; }
  else { c[0] = q / (L * L); c[1] = (q / L) % L; c[2] = q % L; }
  for (int i = 0; i < 3; ++i) c[i] = (L - c[i]) % L;
  return dim == 2 ? c[0] * L + c[1] : (c[0] * L + c[1]) * L + c[2];
}

void orc_brute_rhs(int dim, int L, int n_bands, int n_modes, int n_k_total, int n_q_total,
                   int n_el, const int32_t *el_of_full, const double *eps, const double *hw,
                   const double *g2d, const double *v2d, double sigma_eph, double sigma_pp,
                   double nsigma, double hw_cut, const double *y, double *ydot, int parts) {
  const int N = dim == 2 ? L * L : L * L * L;
  const int n_ph = N * n_modes;
  const double *f = y, *Nq = y + n_el;
  double m;
  for (int i = 0; i < n_el + n_ph; ++i) ydot[i] = 0.0;
  /* I^{e-ph}: electron state nk, sum over m, nu, q */
  if (parts & 1) {
    for (int k = 0; k < N; ++k)
      for (int n = 0; n < n_bands; ++n) {
        int r = el_of_full[k * n_bands + n];
        if (r < 0) continue;
        double sum = 0.0;
        for (int mb = 0; mb < n_bands; ++mb)
          for (int nu = 0; nu < n_modes; ++nu)
            for (int q = 0; q < N; ++q) {
              int s = el_of_full[kplusq(dim, L, k, q) * n_bands + mb];
              if (s < 0) continue;
              int p = q * n_modes + nu;
              if (hw[p] < hw_cut) continue;
              double g2 = g2d[(((size_t)(k * n_bands + n) * n_bands + mb) * n_modes + nu) * N + q];
              if (g2 == 0.0) continue;
              double xe = eps[r] - hw[p] - eps[s], xa = eps[r] + hw[p] - eps[s];
              if (fabs(xe) <= nsigma * sigma_eph)
                sum += g2 * F_em(f[r], f[s], Nq[p], &m) * gauss_delta(xe, sigma_eph);
              if (fabs(xa) <= nsigma * sigma_eph)
                sum += g2 * F_abs(f[r], f[s], Nq[p], &m) * gauss_delta(xa, sigma_eph);
            }
        ydot[r] += -(2.0 * PI_ / HBAR_EV_FS) / (double)n_q_total * sum;
      }
  }
  /* I^{ph-e}: phonon nu q, sum over m, n, k */
  if (parts & 2) {
    for (int q = 0; q < N; ++q)
      for (int nu = 0; nu < n_modes; ++nu) {
        int p = q * n_modes + nu;
        if (hw[p] < hw_cut) continue;
        double sum = 0.0;
        for (int mb = 0; mb < n_bands; ++mb)
          for (int n = 0; n < n_bands; ++n)
            for (int k = 0; k < N; ++k) {
              int r = el_of_full[k * n_bands + n];
              int s = el_of_full[kplusq(dim, L, k, q) * n_bands + mb];
              if (r < 0 || s < 0) continue;
              double g2 = g2d[(((size_t)(k * n_bands + n) * n_bands + mb) * n_modes + nu) * N + q];
              if (g2 == 0.0) continue;
              double xa = eps[r] + hw[p] - eps[s];
              if (fabs(xa) <= nsigma * sigma_eph)
                sum += g2 * F_abs(f[r], f[s], Nq[p], &m) * gauss_delta(xa, sigma_eph);
            }
        ydot[n_el + p] += -(4.0 * PI_ / HBAR_EV_FS) / (double)n_k_total * sum;
      }
  }
  /* I^{ph-ph}: phonon nu q, sum over nu', nu'', q', q'' = -(q+q') */
  if (parts & 4) {
    for (int q = 0; q < N; ++q)
      for (int nu = 0; nu < n_modes; ++nu) {
        int lam = q * n_modes + nu;
        if (hw[lam] < hw_cut) continue;
        double sum = 0.0;
        for (int q1 = 0; q1 < N; ++q1) {
          int q2 = minusq(dim, L, kplusq(dim, L, q, q1));
          for (int n1 = 0; n1 < n_modes; ++n1)
            for (int n2 = 0; n2 < n_modes; ++n2) {
              int a = q1 * n_modes + n1, b = q2 * n_modes + n2;
              if (hw[a] < hw_cut || hw[b] < hw_cut) continue;
              double v2 = v2d[(((size_t)lam * N + q1) * n_modes + n1) * n_modes + n2];
              if (v2 == 0.0) continue;
              double xe = -hw[lam] + hw[a] + hw[b], xa = hw[lam] - hw[a] + hw[b];
              if (fabs(xe) <= nsigma * sigma_pp)
                sum += v2 * G_em(Nq[lam], Nq[a], Nq[b], &m) * gauss_delta(xe, sigma_pp);
              if (fabs(xa) <= nsigma * sigma_pp)
                sum += 2.0 * v2 * G_abs(Nq[lam], Nq[a], Nq[b], &m) * gauss_delta(xa, sigma_pp);
            }
        }
        ydot[n_el + lam] += -(36.0 * PI_ / HBAR_EV_FS) / (double)n_q_total * sum;
      }
  }
}

/* Thread count of the OpenMP loops (timing of the oracle with one thread). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}
