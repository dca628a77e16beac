// Seeded synthetic rt-BTE workloads.
//
// This module builds the *inputs* of the collision-integral problem: the
// momentum grid, band energies eps_nk, phonon energies hbar*omega_nuq, and the
// stored scattering channels with their |g|^2 (e-ph) and |V3|^2 (ph-ph)
// matrix-element values.  It holds none of the method's arithmetic: no delta
// weights, no truncation at n*sigma, no occupation factors, no sums.  Both the
// oracle and the GPU library consume its output; neither is linked into it.
//
// Randomness comes from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11), keyed by the seed and indexed by
// the canonical id of the object it describes, so every value is independent
// of thread count and enumeration order:
//   * |g|^2 is drawn once per unordered e-ph process pair
//     {(nk -> mk+q, nu q), (mk+q -> nk, nu -q)}  (pair symmetry);
//   * |V3|^2 is drawn once per unordered phonon triplet with q+q'+q'' = 0
//     (permutation symmetry), matching the crystal-momentum Kronecker delta of
//     the ph-ph matrix element (Methods, ph-ph matrix element definition).
// A channel is *stored* when its process lies within a shell of half-width
// `shell` around energy conservation (the precomputed scattering matrices only
// hold such channels) and a symmetric hash thinning keeps it.  The shell is
// decided on the canonical orientation of the pair / triplet so that every
// appearance of one process makes the same decision.
#include <cstdint>
#include <cstring>
#include <cmath>
#include <vector>
#include <algorithm>
#include <omp.h>

namespace {

// ---------------------------------------------------------------- Philox4x32-10
struct u32x4 { uint32_t v[4]; };

inline void mulhilo(uint32_t a, uint32_t b, uint32_t &hi, uint32_t &lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  hi = (uint32_t)(p >> 32);
  lo = (uint32_t)p;
}

inline u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo(M0, c.v[0], hi0, lo0);
    mulhilo(M1, c.v[2], hi1, lo1);
    u32x4 n;
    n.v[0] = hi1 ^ c.v[1] ^ k0;
    n.v[1] = lo1;
    n.v[2] = hi0 ^ c.v[3] ^ k1;
    n.v[3] = lo0;
    c = n;
  }
  return c;
}

inline double u01(uint32_t x) { return ((double)x + 0.5) * (1.0 / 4294967296.0); }

// Standard normal from two uniforms (Box-Muller).
inline double normal01(uint32_t a, uint32_t b) {
  const double two_pi = 6.283185307179586476925286766559;
  return std::sqrt(-2.0 * std::log(u01(a))) * std::cos(two_pi * u01(b));
}

enum : uint32_t { STREAM_EPH = 0x65706831u, STREAM_PP = 0x70707033u };

// Thinning decisions use the splitmix64 finalizer (Steele, Lea, Flood,
// OOPSLA'14) of the packed canonical id: cheap enough to run on every
// candidate inside the shell.  Philox supplies the values of kept channels.
inline double keep_u01(uint64_t packed, uint64_t seed) {
  uint64_t z = packed + seed * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return ((double)(z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

}  // namespace

extern "C" {

// ------------------------------------------------------------------- params
typedef struct {
  int32_t dim;        // 2 or 3
  int32_t L;          // grid points per reciprocal-lattice axis (k and q share it)
  int32_t lattice;    // 0 square (cos tight binding), 1 triangular (graphene-like),
                      // 2 simple cubic (silicon-like conduction bands)
  int32_t n_bands;    // electron bands
  int32_t n_modes;    // phonon branches
  int32_t with_eph, with_pp;
  int32_t quantize;   // 1: round every energy to a multiple of `quantum`
  double quantum;     // eV
  double t_hop;       // eV, band hopping
  double win_lo, win_hi;           // electron energy window (eV)
  double shell_eph, shell_pp;      // stored-channel shell half-width (eV)
  double keep_eph, keep_pp;        // symmetric thinning probabilities
  double g2_mu, g2_sig;            // ln|g|^2 ~ N(mu, sig), |g|^2 in eV^2
  double v2_mu, v2_sig;            // ln|V3|^2 ~ N(mu, sig), eV^2
  uint64_t seed;
  double keep_pp_q;                // symmetric thinning of q-point triplets (q, q', q''),
                                   // decided before any branch: 1 keeps all
} synth_params;

void synth_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  u32x4 c{{ctr[0], ctr[1], ctr[2], ctr[3]}};
  u32x4 r = philox4x32_10(c, key[0], key[1]);
  for (int i = 0; i < 4; ++i) out[i] = r.v[i];
}

}  // extern "C"

namespace {

struct Grid {
  int dim, L, N;
  std::vector<int32_t> c0, c1, c2, negt;  // component tables and -k table
  void init(int d, int l) {
    dim = d; L = l; N = d == 2 ? l * l : l * l * l;
    c0.resize(N); c1.resize(N); c2.resize(N); negt.resize(N);
    for (int i = 0; i < N; ++i) {
      int c[3];
      if (dim == 2) { c[0] = i / L; c[1] = i % L; c[2] = 0; }
      else { c[0] = i / (L * L); c[1] = (i / L) % L; c[2] = i % L; }
      c0[i] = c[0]; c1[i] = c[1]; c2[i] = c[2];
    }
    for (int i = 0; i < N; ++i) {
      int c[3] = {(L - c0[i]) % L, (L - c1[i]) % L, (L - c2[i]) % L};
      negt[i] = index(c);
    }
  }
  void comp(int idx, int c[3]) const { c[0] = c0[idx]; c[1] = c1[idx]; c[2] = c2[idx]; }
  int index(const int c[3]) const {
    return dim == 2 ? c[0] * L + c[1] : (c[0] * L + c[1]) * L + c[2];
  }
  int add(int a, int b) const {
    int x = c0[a] + c0[b]; x -= x >= L ? L : 0;
    int y = c1[a] + c1[b]; y -= y >= L ? L : 0;
    if (dim == 2) return x * L + y;
    int z = c2[a] + c2[b]; z -= z >= L ? L : 0;
    return (x * L + y) * L + z;
  }
  int neg(int a) const { return negt[a]; }
  // canonical representative of {k, -k}
  int rep(int a) const { return std::min(a, neg(a)); }
};

const double TWO_PI = 6.283185307179586476925286766559;

double band_energy(const synth_params &p, const Grid &g, int k, int n) {
  int c[3];
  g.comp(g.rep(k), c);
  double th[3];
  for (int i = 0; i < 3; ++i) th[i] = TWO_PI * c[i] / p.L;
  double e = 0.0;
  if (p.lattice == 0) {
    double s = std::cos(th[0]) + std::cos(th[1]);
    e = (n % 2 == 0 ? -2.0 : 2.0) * p.t_hop * s;
  } else if (p.lattice == 1) {
    double g2 = 3.0 + 2.0 * std::cos(th[0]) + 2.0 * std::cos(th[1]) + 2.0 * std::cos(th[0] - th[1]);
    double mag = std::sqrt(std::max(g2, 0.0));
    e = (n % 2 == 0 ? -1.0 : 1.0) * p.t_hop * mag;
  } else {
    static const double offs[4] = {0.0, 0.045, 0.11, 0.18};
    static const double mass[4] = {1.0, 0.8, 1.25, 0.65};
    double s = 0.0;
    for (int i = 0; i < 3; ++i) s += 1.0 - std::cos(th[i]);
    e = offs[n % 4] + mass[n % 4] * p.t_hop * s;
  }
  if (p.quantize) e = p.quantum * std::nearbyint(e / p.quantum);
  return e;
}

double phonon_energy(const synth_params &p, const Grid &g, int q, int nu) {
  int c[3];
  g.comp(g.rep(q), c);
  double th[3];
  for (int i = 0; i < 3; ++i) th[i] = TWO_PI * c[i] / p.L;
  double w = 0.0;  // meV
  if (p.lattice == 0) {
    static const double lo[3] = {20.0, 60.0, 110.0}, hi[3] = {60.0, 110.0, 160.0};
    double s = (2.0 - std::cos(th[0]) - std::cos(th[1])) / 4.0;
    w = lo[nu % 3] + (hi[nu % 3] - lo[nu % 3]) * s;
  } else if (p.lattice == 1) {
    double g2 = 3.0 + 2.0 * std::cos(th[0]) + 2.0 * std::cos(th[1]) + 2.0 * std::cos(th[0] - th[1]);
    double s = std::min(std::max((9.0 - g2) / 9.0, 0.0), 1.0);
    switch (nu % 6) {
      case 0: w = 65.0 * s; break;                  // ZA
      case 1: w = 125.0 * std::sqrt(s); break;      // TA
      case 2: w = 160.0 * std::sqrt(s); break;      // LA
      case 3: w = 110.0 - 43.0 * s; break;          // ZO
      case 4: w = 196.0 - 46.0 * s; break;          // TO
      default: w = 194.0 - 34.0 * s; break;         // LO
    }
  } else {
    double s = 0.0;
    for (int i = 0; i < 3; ++i) { double h = std::sin(0.5 * th[i]); s += h * h; }
    s /= 3.0;
    switch (nu % 6) {
      case 0: w = 25.0 * std::sqrt(s); break;       // TA1
      case 1: w = 27.0 * std::sqrt(s); break;       // TA2
      case 2: w = 60.0 * std::sqrt(s); break;       // LA
      case 3: w = 64.0 - 4.0 * s; break;            // TO1
      case 4: w = 63.0 - 3.0 * s; break;            // TO2
      default: w = 62.0 - 2.0 * s; break;           // LO
    }
  }
  w *= 1e-3;  // eV
  if (p.quantize) w = p.quantum * std::max(1.0, std::nearbyint(w / p.quantum));
  return w;
}

struct Model {
  synth_params p;
  Grid g;
  int n_full_el;                 // n_bands * N
  std::vector<double> eps_full;  // [k*n_bands + n]
  std::vector<int32_t> el_of_full;   // full id -> windowed id or -1
  std::vector<int32_t> full_of_el;   // windowed id -> full id
  std::vector<double> hw;        // [q*n_modes + nu]
  uint32_t k0, k1;
  // stored channels, enumerated once, kept per chunk of consecutive rows
  struct Chunk { std::vector<int32_t> row, i1, i2; std::vector<double> val; };
  std::vector<Chunk> eph_chunks, pp_chunks;
  int64_t n_eph = 0, n_pp = 0;
};

const int ROWS_PER_CHUNK = 16;

// Time reversal: the image of a state under k -> -k (the same band or branch).
inline int inv_el(const Model &m, int f) {
  const int nb = m.p.n_bands;
  return m.g.neg(f / nb) * nb + f % nb;
}
inline int inv_ph(const Model &m, int l) {
  const int nm = m.p.n_modes;
  return m.g.neg(l / nm) * nm + l % nm;
}

// Sorted ids of a triplet or of its time-reversed image, whichever is
// lexicographically smaller: the key every random decision about the
// triplet is drawn from, so |V3|^2 and the thinning are the same for a
// triplet in any order and for its image (real crystals have time-reversal
// symmetry, which keeps N even in q and the carrier number conserved).
inline void canon3(int a, int b, int c, int ia, int ib, int ic, int out[3]) {
  int x[3] = {a, b, c}, y[3] = {ia, ib, ic};
  std::sort(x, x + 3);
  std::sort(y, y + 3);
  const bool use_y = std::lexicographical_compare(y, y + 3, x, x + 3);
  for (int i = 0; i < 3; ++i) out[i] = use_y ? y[i] : x[i];
}

// Is the unordered e-ph pair stored, and with which |g|^2?  Decided on the
// canonical orientation (lower full id first) so both directions agree, and
// keyed on the smaller of the pair and its time-reversed image.
inline bool pair_channel(const Model &m, int f_lo, int f_hi, int nu, int q_lo_to_hi, double *g2) {
  const synth_params &p = m.p;
  double w = m.hw[(size_t)q_lo_to_hi * p.n_modes + nu];
  double e_lo = m.eps_full[f_lo], e_hi = m.eps_full[f_hi];
  double x1 = std::fabs(e_lo - w - e_hi), x2 = std::fabs(e_lo + w - e_hi);
  if (std::min(x1, x2) > p.shell_eph) return false;
  int k_lo = f_lo, k_hi = f_hi;
  {
    const int a = inv_el(m, f_lo), b = inv_el(m, f_hi);
    const int i_lo = std::min(a, b), i_hi = std::max(a, b);
    if (i_lo < k_lo || (i_lo == k_lo && i_hi < k_hi)) { k_lo = i_lo; k_hi = i_hi; }
  }
  if (p.keep_eph < 1.0) {
    uint64_t packed = (uint64_t)k_lo | ((uint64_t)k_hi << 21) | ((uint64_t)nu << 42) | (1ull << 50);
    if (!(keep_u01(packed, p.seed) < p.keep_eph)) return false;
  }
  u32x4 c{{(uint32_t)k_lo, (uint32_t)k_hi, (uint32_t)nu, STREAM_EPH}};
  u32x4 r = philox4x32_10(c, m.k0, m.k1);
  *g2 = std::exp(p.g2_mu + p.g2_sig * normal01(r.v[1], r.v[2]));
  return true;
}

// Is the q-point triplet (q0, q1, q2), q0 + q1 + q2 = 0, kept by the
// q-level thinning?  Decided on the canonical sorted ids: the same for every
// ordering and for the time-reversed triplet.
inline bool qtriplet_kept(const Model &m, int q0, int q1, int q2) {
  if (!(m.p.keep_pp_q < 1.0)) return true;
  int id[3];
  canon3(q0, q1, q2, m.g.neg(q0), m.g.neg(q1), m.g.neg(q2), id);
  uint64_t packed = (uint64_t)id[0] | ((uint64_t)id[1] << 21) | ((uint64_t)id[2] << 42) | (1ull << 62);
  return keep_u01(packed, m.p.seed) < m.p.keep_pp_q;
}

// Is the unordered phonon triplet stored, and with which |V3|^2?  The shell
// test uses the sorted frequencies, the hash the canonical sorted ids: both
// are invariant under permutation of the three phonons and under time
// reversal.
inline bool triplet_channel(const Model &m, int l0, int l1, int l2, double *v2) {
  const synth_params &p = m.p;
  const int nm = p.n_modes;
  if (!qtriplet_kept(m, l0 / nm, l1 / nm, l2 / nm)) return false;
  const double wa = m.hw[l0], wb = m.hw[l1], wc = m.hw[l2];
  const double hi = std::max(std::max(wa, wb), wc), lo = std::min(std::min(wa, wb), wc);
  const double mid = std::max(std::min(wa, wb), std::min(std::max(wa, wb), wc));
  if (!(std::fabs(hi - (mid + lo)) <= p.shell_pp)) return false;
  int id[3];
  canon3(l0, l1, l2, inv_ph(m, l0), inv_ph(m, l1), inv_ph(m, l2), id);
  if (p.keep_pp < 1.0) {
    uint64_t packed = (uint64_t)id[0] | ((uint64_t)id[1] << 21) | ((uint64_t)id[2] << 42) | (1ull << 63);
    if (!(keep_u01(packed, p.seed) < p.keep_pp)) return false;
  }
  u32x4 c{{(uint32_t)id[0], (uint32_t)id[1], (uint32_t)id[2], STREAM_PP}};
  u32x4 r = philox4x32_10(c, m.k0, m.k1);
  *v2 = std::exp(p.v2_mu + p.v2_sig * normal01(r.v[1], r.v[2]));
  return true;
}

// Visit the stored e-ph channels of windowed electron row r, in (q, m, nu) order.
template <class F>
void eph_row(const Model &m, int r, F &&emit) {
  const synth_params &p = m.p;
  int fr = m.full_of_el[r];
  int k = fr / p.n_bands;
  for (int q = 0; q < m.g.N; ++q) {
    int kq = m.g.add(k, q);
    int mq = m.g.neg(q);
    for (int mb = 0; mb < p.n_bands; ++mb) {
      int fs = kq * p.n_bands + mb;
      int s = m.el_of_full[fs];
      if (s < 0) continue;
      for (int nu = 0; nu < p.n_modes; ++nu) {
        double g2;
        bool ok = fr <= fs ? pair_channel(m, fr, fs, nu, q, &g2)
                           : pair_channel(m, fs, fr, nu, mq, &g2);
        if (ok) emit(s, q * p.n_modes + nu, g2);
      }
    }
  }
}

// Visit the stored ph-ph channels of phonon row lam = q*n_modes + nu, in
// (q', nu', nu'') order, with q'' = -(q + q').
template <class F>
void pp_row(const Model &m, int lam, F &&emit) {
  const synth_params &p = m.p;
  const int nm = p.n_modes;
  int q = lam / nm;
  int mq = m.g.neg(q);
  const double w0 = m.hw[lam];
  for (int q1 = 0; q1 < m.g.N; ++q1) {
    int q2 = m.g.add(mq, m.g.neg(q1));
    if (!qtriplet_kept(m, q, q1, q2)) continue;   // the same decision triplet_channel takes
    const double *w1 = &m.hw[(size_t)q1 * nm], *w2 = &m.hw[(size_t)q2 * nm];
    // branch-free shell test of all (n1, n2) first (same selection as
    // triplet_channel), then the full decision for the few that pass
    uint64_t pass = 0;
    for (int n1 = 0; n1 < nm; ++n1)
      for (int n2 = 0; n2 < nm; ++n2) {
        const double a = w0, b = w1[n1], c = w2[n2];
        const double hi = std::max(std::max(a, b), c), lo = std::min(std::min(a, b), c);
        const double mid = std::max(std::min(a, b), std::min(std::max(a, b), c));
        pass |= (uint64_t)(std::fabs(hi - (mid + lo)) <= p.shell_pp) << (n1 * nm + n2);
      }
    while (pass) {
      const int bit = __builtin_ctzll(pass);
      pass &= pass - 1;
      const int n1 = bit / nm, n2 = bit % nm;
      const int a = q1 * nm + n1, b = q2 * nm + n2;
      double v2;
      if (triplet_channel(m, lam, a, b, &v2)) emit(a, b, v2);
    }
  }
}

}  // namespace

extern "C" {

void *synth_create(const synth_params *pp) {
  Model *m = new Model();
  m->p = *pp;
  const synth_params &p = m->p;
  m->g.init(p.dim, p.L);
  m->k0 = (uint32_t)(p.seed & 0xffffffffu);
  m->k1 = (uint32_t)(p.seed >> 32);
  const int N = m->g.N;
  m->n_full_el = p.n_bands * N;
  m->eps_full.resize(m->n_full_el);
  m->el_of_full.assign(m->n_full_el, -1);
  for (int k = 0; k < N; ++k)
    for (int n = 0; n < p.n_bands; ++n) {
      double e = band_energy(p, m->g, k, n);
      m->eps_full[k * p.n_bands + n] = e;
    }
  for (int f = 0; f < m->n_full_el; ++f) {
    double e = m->eps_full[f];
    if (e >= p.win_lo && e <= p.win_hi) {
      m->el_of_full[f] = (int32_t)m->full_of_el.size();
      m->full_of_el.push_back(f);
    }
  }
  m->hw.resize((size_t)N * p.n_modes);
  for (int q = 0; q < N; ++q)
    for (int nu = 0; nu < p.n_modes; ++nu) m->hw[(size_t)q * p.n_modes + nu] = phonon_energy(p, m->g, q, nu);

  const int n_el = (int)m->full_of_el.size();
  const int n_ph = N * p.n_modes;
  if (p.with_eph) {
    const int nc = (n_el + ROWS_PER_CHUNK - 1) / ROWS_PER_CHUNK;
    m->eph_chunks.resize(nc);
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < nc; ++c) {
      Model::Chunk &ch = m->eph_chunks[c];
      for (int r = c * ROWS_PER_CHUNK; r < std::min(n_el, (c + 1) * ROWS_PER_CHUNK); ++r)
        eph_row(*m, r, [&](int s, int ph, double g) {
          ch.row.push_back(r); ch.i1.push_back(s); ch.i2.push_back(ph); ch.val.push_back(g);
        });
    }
  }
  if (p.with_pp) {
    const int nc = (n_ph + ROWS_PER_CHUNK - 1) / ROWS_PER_CHUNK;
    m->pp_chunks.resize(nc);
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < nc; ++c) {
      Model::Chunk &ch = m->pp_chunks[c];
      for (int l = c * ROWS_PER_CHUNK; l < std::min(n_ph, (c + 1) * ROWS_PER_CHUNK); ++l)
        pp_row(*m, l, [&](int aa, int bb, double v) {
          ch.row.push_back(l); ch.i1.push_back(aa); ch.i2.push_back(bb); ch.val.push_back(v);
        });
    }
  }
  for (auto &c : m->eph_chunks) m->n_eph += (int64_t)c.row.size();
  for (auto &c : m->pp_chunks) m->n_pp += (int64_t)c.row.size();
  return m;
}

void synth_destroy(void *h) { delete (Model *)h; }

// sizes[0..5] = n_el, n_ph, N (grid points), n_eph, n_pp, n_full_el
void synth_sizes(const void *h, int64_t sizes[6]) {
  const Model *m = (const Model *)h;
  sizes[0] = (int64_t)m->full_of_el.size();
  sizes[1] = (int64_t)m->g.N * m->p.n_modes;
  sizes[2] = m->g.N;
  sizes[3] = m->n_eph;
  sizes[4] = m->n_pp;
  sizes[5] = m->n_full_el;
}

// Per-state data. eps[n_el], el_k[n_el], el_band[n_el], hw[n_ph],
// el_of_full[n_full_el] (windowed id or -1).
void synth_states(const void *h, double *eps, int32_t *el_k, int32_t *el_band, double *hw,
                  int32_t *el_of_full) {
  const Model *m = (const Model *)h;
  const int nb = m->p.n_bands;
  for (size_t r = 0; r < m->full_of_el.size(); ++r) {
    int f = m->full_of_el[r];
    eps[r] = m->eps_full[f];
    el_k[r] = f / nb;
    el_band[r] = f % nb;
  }
  std::memcpy(hw, m->hw.data(), m->hw.size() * sizeof(double));
  std::memcpy(el_of_full, m->el_of_full.data(), m->el_of_full.size() * sizeof(int32_t));
}

}  // extern "C"

namespace {
void copy_chunks(std::vector<Model::Chunk> &chunks, int32_t *row, int32_t *i1, int32_t *i2, double *val) {
  std::vector<int64_t> off(chunks.size() + 1, 0);
  for (size_t c = 0; c < chunks.size(); ++c) off[c + 1] = off[c] + (int64_t)chunks[c].row.size();
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c = 0; c < (int64_t)chunks.size(); ++c) {
    Model::Chunk &ch = chunks[c];
    size_t n = ch.row.size();
    if (n) {
      std::memcpy(row + off[c], ch.row.data(), n * sizeof(int32_t));
      std::memcpy(i1 + off[c], ch.i1.data(), n * sizeof(int32_t));
      std::memcpy(i2 + off[c], ch.i2.data(), n * sizeof(int32_t));
      std::memcpy(val + off[c], ch.val.data(), n * sizeof(double));
    }
    Model::Chunk().row.swap(ch.row);  // release as we go
    std::vector<int32_t>().swap(ch.i1);
    std::vector<int32_t>().swap(ch.i2);
    std::vector<double>().swap(ch.val);
  }
}
}  // namespace

extern "C" {

// Stored e-ph channels, grouped by electron row in row order (within a row:
// q, then final band, then mode).  Single use: releases the enumeration.
void synth_fill_eph(void *h, int32_t *row, int32_t *partner, int32_t *phonon, double *g2) {
  copy_chunks(((Model *)h)->eph_chunks, row, partner, phonon, g2);
}

// Stored ph-ph channels, grouped by phonon row in row order (within a row:
// q', then nu', then nu'').  Single use: releases the enumeration.
void synth_fill_pp(void *h, int32_t *row, int32_t *a, int32_t *b, double *v2) {
  copy_chunks(((Model *)h)->pp_chunks, row, a, b, v2);
}

// Dense matrix-element tables for tiny grids (brute-force sums).  Zero where
// no channel is stored.
//   g2d[((f_r * n_bands + m) * n_modes + nu) * N + q]  for every full-grid
//       electron state f_r = k*n_bands+n, final band m, mode nu, phonon q
//       (final state m, k+q);
//   v2d[((lam * N + q1) * n_modes + n1) * n_modes + n2]  for phonon row lam,
//       partner (n1, q1) and (n2, -(q+q1)).
void synth_dense(const void *h, double *g2d, double *v2d) {
  const Model *m = (const Model *)h;
  const synth_params &p = m->p;
  const int N = m->g.N, nb = p.n_bands, nm = p.n_modes;
  if (g2d) {
    for (int fr = 0; fr < m->n_full_el; ++fr) {
      int k = fr / nb;
      for (int mb = 0; mb < nb; ++mb)
        for (int nu = 0; nu < nm; ++nu)
          for (int q = 0; q < N; ++q) {
            int fs = m->g.add(k, q) * nb + mb;
            double g2 = 0.0;
            bool ok = fr <= fs ? pair_channel(*m, fr, fs, nu, q, &g2)
                               : pair_channel(*m, fs, fr, nu, m->g.neg(q), &g2);
            g2d[(((size_t)fr * nb + mb) * nm + nu) * N + q] = (ok && p.with_eph) ? g2 : 0.0;
          }
    }
  }
  if (v2d) {
    for (int lam = 0; lam < N * nm; ++lam) {
      int q = lam / nm;
      for (int q1 = 0; q1 < N; ++q1) {
        int q2 = m->g.neg(m->g.add(q, q1));
        for (int n1 = 0; n1 < nm; ++n1)
          for (int n2 = 0; n2 < nm; ++n2) {
            double v2 = 0.0;
            bool ok = triplet_channel(*m, lam, q1 * nm + n1, q2 * nm + n2, &v2);
            v2d[(((size_t)lam * N + q1) * nm + n1) * nm + n2] = (ok && p.with_pp) ? v2 : 0.0;
          }
      }
    }
  }
}

int synth_threads(void) { return omp_get_max_threads(); }
void synth_set_threads(int n) { omp_set_num_threads(n); }

}  // extern "C"
