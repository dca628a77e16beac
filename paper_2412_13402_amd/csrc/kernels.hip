// HIP kernels for gfx950: collision integrals over destination-sorted channel
// lists, ERK stage updates, WRMS reduction, step control, and the create-time
// channel preparation.
//
// Collision integrals (Methods, Eq. (e-ph) and Eq. (ph-ph)).  Destination rows
// of y' form groups of up to 16 consecutive rows of one kind; a group's
// channels are cut into work items of bounded length, each streamed once by
// one wavefront with non-temporal loads (FP64: 16 bytes per channel, or 12 in
// the packed layout; mixed precision: 8 or 10), laid out so that every load
// instruction of a wavefront reads whole lines.  The group's channels are stored
// merged in partner order, so rows that share partners (the modes of one
// phonon wave vector; neighbouring electron k-points) gather their
// populations from the same cache lines at the same time.  Each lane keeps
// one accumulator per row of the group in its own LDS slots; the slots are
// summed in a fixed order at the end, with no atomics, so results are
// deterministic.  Groups are visited longest first,
// so long groups never straggle at the end of the grid.
#include "internal.h"

#include <algorithm>

namespace rtbte {

typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4i ld_stream(const Channel* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const v4i*>(p));
}

__device__ __forceinline__ double chan_w(const v4i c) { return __hiloint2double(c.w, c.z); }

enum { K_EPH = 0, K_PHE = 1, K_PP = 2 };

// Occupation factors (Methods, after Eq. (e-ph) and Eq. (ph-ph)), each as
// gain - loss.  Row invariants (x, 1-x or N, N+1) are passed precomputed.
//   e-ph, electron row r, partner s, phonon p:
//     F_em  = f_r (1-f_s)(1+N_p) - (1-f_r) f_s N_p
//     F_abs = f_r (1-f_s) N_p    - (1-f_r) f_s (1+N_p)
//   ph-e, phonon row p, electrons r, s:  F_abs(f_r, f_s, N_p)
//   ph-ph, phonon row l, partners a, b:
//     G_em  = N (N_a+1)(N_b+1) - (N+1) N_a N_b
//     G_abs = N (N_a+1) N_b    - (N+1) N_a (N_b+1)
// With DERIV the term is -w dF/dx_r instead, the derivative of the factor
// with respect to the row's own population x_r (partners held fixed): the
// row's sum then negates to the linearized (relaxation-time) rate.  Each
// factor is x_r X - x_r' Y with x_r' = 1 - x_r (electron rows) or x_r + 1
// (phonon rows), so dF/dx_r = X + Y or X - Y.
template <int KIND, bool DERIV = false>
__device__ __forceinline__ double term_w(bool em, double w, double g0, double g1, double xr, double xr1) {
  if (KIND == K_EPH) {            // xr = f_r, xr1 = 1 - f_r, g0 = f_s, g1 = N_p
    const double n1 = g1 + 1.0;
    const double X = (1.0 - g0) * (em ? n1 : g1), Y = g0 * (em ? g1 : n1);
    if (DERIV) return -w * (X + Y);
    return w * (xr * X - xr1 * Y);
  } else if (KIND == K_PHE) {     // xr = N_p, xr1 = N_p + 1, g0 = f_r, g1 = f_s
    const double X = g0 * (1.0 - g1), Y = (1.0 - g0) * g1;
    if (DERIV) return -w * (X - Y);
    return w * (X * xr - Y * xr1);
  } else {                        // xr = N, xr1 = N + 1, g0 = N_a, g1 = N_b
    const double b1 = g1 + 1.0;
    const double X = (g0 + 1.0) * (em ? b1 : g1), Y = g0 * (em ? g1 : b1);
    if (DERIV) return -w * (X - Y);
    return w * (xr * X - xr1 * Y);
  }
}

template <int KIND, bool DERIV>
__device__ __forceinline__ double term(const v4i c, double g0, double g1, double xr, double xr1) {
  return term_w<KIND, DERIV>(c.y < 0, chan_w(c), g0, g1, xr, xr1);
}

// Per-lane accumulators of one wavefront: one slot per (row of the group,
// lane), so every lane adds only to its own slots (in a fixed order: the
// sums stay deterministic) without per-row selects in registers.
template <int G>
struct LaneAcc {
  double* slot;   // this lane's first slot; row j at slot[64 * j]
  double reg;     // G == 1: the accumulator itself
  __device__ __forceinline__ void add(int tag, double v) {
    if (G == 1) reg += v;
    else slot[64 * tag] += v;
  }
};

// One channel: w * factor with the gathered partner populations g0, g1 and
// the row's own population (kept in LDS), added to the accumulator of its row.
template <int G, int KIND, bool DERIV>
__device__ __forceinline__ void chan_acc(LaneAcc<G>& acc, const v4i c, double g0, double g1,
                                         const double* rowv) {
  const int tag = G == 1 ? 0 : ((c.x >> kTagShift) & 15);
  const double xr = rowv[tag];
  const double xr1 = KIND == K_EPH ? 1.0 - xr : xr + 1.0;
  acc.add(tag, term<KIND, DERIV>(c, g0, g1, xr, xr1));
}

// Stream [s, e) with a two-stage software pipeline: the gathers of batch k
// are issued before the stream loads of batch k+1, so waiting for the
// gathers (in-order completion counters) leaves the next batch in flight.
template <int G, int LANES, int KIND, bool DERIV>
__device__ __forceinline__ void seg_sum(LaneAcc<G>& acc, const Channel* __restrict__ ch, int64_t s,
                                        int64_t e, int lane, const double* __restrict__ z,
                                        const double* rowv) {
  constexpr int64_t STEP = 4 * LANES;
  int64_t i = s + lane;
  if (i + 3 * LANES < e) {
    v4i c0 = ld_stream(ch + i), c1 = ld_stream(ch + i + LANES);
    v4i c2 = ld_stream(ch + i + 2 * LANES), c3 = ld_stream(ch + i + 3 * LANES);
    i += STEP;
    for (;;) {
      const double a0 = z[c0.x & kPosMask], b0 = z[c0.y & kPosMask];
      const double a1 = z[c1.x & kPosMask], b1 = z[c1.y & kPosMask];
      const double a2 = z[c2.x & kPosMask], b2 = z[c2.y & kPosMask];
      const double a3 = z[c3.x & kPosMask], b3 = z[c3.y & kPosMask];
      const bool more = i + 3 * LANES < e;
      v4i n0 = c0, n1 = c1, n2 = c2, n3 = c3;
      if (more) {
        n0 = ld_stream(ch + i);
        n1 = ld_stream(ch + i + LANES);
        n2 = ld_stream(ch + i + 2 * LANES);
        n3 = ld_stream(ch + i + 3 * LANES);
      }
      chan_acc<G, KIND, DERIV>(acc, c0, a0, b0, rowv);
      chan_acc<G, KIND, DERIV>(acc, c1, a1, b1, rowv);
      chan_acc<G, KIND, DERIV>(acc, c2, a2, b2, rowv);
      chan_acc<G, KIND, DERIV>(acc, c3, a3, b3, rowv);
      if (!more) break;
      c0 = n0; c1 = n1; c2 = n2; c3 = n3;
      i += STEP;
    }
  }
  for (; i < e; i += LANES) {
    const v4i c = ld_stream(ch + i);
    chan_acc<G, KIND, DERIV>(acc, c, z[c.x & kPosMask], z[c.y & kPosMask], rowv);
  }
}

typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

// One packed FP64 channel: the 8-byte word (lo, hi) and the low weight word
// wl (layout in internal.h; 32-bit operations only), the gathered partner
// values g0, g1.
template <int G, int KIND, bool DERIV>
__device__ __forceinline__ void chan_p12(LaneAcc<G>& acc, uint32_t lo, uint32_t hi, uint32_t wl, double g0,
                                         double g1, const double* rowv, int P, int sh) {
  const int tag = G == 1 ? 0 : (int)((lo >> P) & 15u);
  const bool em = (hi >> P) & 1u;
  const uint32_t wh = (lo >> (P + 4)) | ((hi >> (P + 1)) << (28 - P));   // field bits 32.. (exponent, top mantissa)
  const uint32_t h32 = sh ? __builtin_amdgcn_alignbit(wh, wl, 32 - sh) : wh;
  const double w = __hiloint2double((int)h32, (int)(wl << sh));
  const double xr = rowv[tag];
  const double xr1 = KIND == K_EPH ? 1.0 - xr : xr + 1.0;
  acc.add(tag, term_w<KIND, DERIV>(em, w, g0, g1, xr, xr1));
}

// Channels [s, e) of one kind from the packed FP64 stream in batches of one
// 256-channel tile: the words are read as channel pairs (16 B), lanes on
// consecutive pairs, two pairs 64 apart per lane, and the low weight words of
// a lane's four channels as one 16-byte load (the tile-permuted order written
// by k_pack12), so every load instruction covers whole lines; two-stage
// pipeline as in seg_sum.  Batches start on tile boundaries (channels before
// s are masked off; tiles never straddle instances).  `off` is the
// instance's offset in z.
template <int G, int KIND, bool DERIV>
__device__ __forceinline__ void seg_sum_p12(LaneAcc<G>& acc, const RowArgs& a, int64_t s, int64_t e, int lane,
                                            const double* __restrict__ z, const double* rowv, uint32_t off) {
  if (s >= e) return;
  const v4u* A2 = reinterpret_cast<const v4u*>(a.pk);
  const v4u* B4 = reinterpret_cast<const v4u*>(a.pkw);
  const int P = a.pack_p, sh = 52 - a.pack_m;
  const uint32_t pmask = (1u << P) - 1u;
  const int64_t p_end = (e + 1) / 2;           // pairs [s / 2, p_end)
  int64_t pb = (s / 2) & ~(int64_t)127;        // first pair of the batch (wave-uniform, tile-aligned)
  v4u c[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int64_t q = pb + lane + 64 * j;
    c[j] = v4u{0u, 0u, 0u, 0u};
    if (q < p_end) c[j] = __builtin_nontemporal_load(A2 + q);
  }
  v4u wl = __builtin_nontemporal_load(B4 + pb / 2 + lane);   // the tile is allocated whole
  for (;;) {
    double g0[4], g1[4];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      g0[2 * j] = z[(c[j].x & pmask) + off];
      g1[2 * j] = z[(c[j].y & pmask) + off];
      g0[2 * j + 1] = z[(c[j].z & pmask) + off];
      g1[2 * j + 1] = z[(c[j].w & pmask) + off];
    }
    const int64_t nb = pb + 128;
    const bool more = nb < p_end;
    v4u n[2];
    v4u m = v4u{0u, 0u, 0u, 0u};
#pragma unroll
    for (int j = 0; j < 2; ++j) n[j] = v4u{0u, 0u, 0u, 0u};
    if (more) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int64_t q = nb + lane + 64 * j;
        if (q < p_end) n[j] = __builtin_nontemporal_load(A2 + q);
      }
      m = __builtin_nontemporal_load(B4 + nb / 2 + lane);
    }
    const uint32_t wlo[4] = {wl.x, wl.y, wl.z, wl.w};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t ca = 2 * (pb + lane + 64 * j);
      if (ca >= s && ca < e)
        chan_p12<G, KIND, DERIV>(acc, c[j].x, c[j].y, wlo[2 * j], g0[2 * j], g1[2 * j], rowv, P, sh);
      if (ca + 1 >= s && ca + 1 < e)
        chan_p12<G, KIND, DERIV>(acc, c[j].z, c[j].w, wlo[2 * j + 1], g0[2 * j + 1], g1[2 * j + 1], rowv, P, sh);
    }
    if (!more) break;
#pragma unroll
    for (int j = 0; j < 2; ++j) c[j] = n[j];
    wl = m;
    pb = nb;
  }
}

// Gaussian delta of the truncated sums (the same function the create-time
// channel preparation evaluates).
__device__ __forceinline__ double gdelta(double x, double sigma) {
  const double u = x / sigma;
  return exp(-u * u) / (sigma * kSqrtPi);
}

// ------------------------------------------------- matrix-free ph-ph weights
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of
// (c0, c1, c2, c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
// lo(M0 c0)), the key bumped by the Weyl constants after every round.
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// n / d for n < 2^31 and d >= 1 from the FP64 reciprocal rd = 1/d: the
// truncated product is exact or, when n is a multiple of d, one short (its
// relative error is below 2^-51, so it can never reach the next integer),
// and one correction step makes it exact.
__device__ __forceinline__ uint32_t div_rcp(uint32_t n, uint32_t d, double rd) {
  uint32_t q = (uint32_t)((double)n * rd);
  if (n - q * d >= d) ++q;
  return q;
}

// -i mod L for 0 <= i < L
__device__ __forceinline__ uint32_t neg_mod(uint32_t i, uint32_t L) { return i ? L - i : 0u; }

// Time-reversed phonon state: -q on the periodic grid, the same branch.
__device__ __forceinline__ uint32_t reversed_phonon(uint32_t id, const PpModel& m) {
  const uint32_t nm = (uint32_t)m.n_modes, L = (uint32_t)m.L;
  const uint32_t q = div_rcp(id, nm, m.rcp_modes), nu = id - q * nm;
  uint32_t nq;
  if (m.dim == 2) {
    const uint32_t i = div_rcp(q, L, m.rcp_L), j = q - i * L;
    nq = neg_mod(i, L) * L + neg_mod(j, L);
  } else {
    const uint32_t t = div_rcp(q, L, m.rcp_L), k = q - t * L;   // t = i L + j
    const uint32_t i = div_rcp(t, L, m.rcp_L), j = t - i * L;
    nq = (neg_mod(i, L) * L + neg_mod(j, L)) * L + neg_mod(k, L);
  }
  return nq * nm + nu;
}

__device__ __forceinline__ void sort3(uint32_t& a, uint32_t& b, uint32_t& c) {
  uint32_t t;
  if (a > b) { t = a; a = b; b = t; }
  if (b > c) { t = b; b = c; c = t; }
  if (a > b) { t = a; a = b; b = t; }
}

// ln |V3|^2 of the triplet (phonon ids l, a, b) under the model
// (rtbte_pp_model): ln_mu + ln_sigma * (Box-Muller normal of the Philox draw).
__device__ __forceinline__ double model_ln_v2(const PpModel& m, uint32_t l, uint32_t a, uint32_t b) {
  uint32_t x0 = l, x1 = a, x2 = b;
  uint32_t y0 = reversed_phonon(l, m), y1 = reversed_phonon(a, m), y2 = reversed_phonon(b, m);
  sort3(x0, x1, x2);
  sort3(y0, y1, y2);
  const bool rev = y0 < x0 || (y0 == x0 && (y1 < x1 || (y1 == x1 && y2 < x2)));
  const uint4 r = philox10(rev ? make_uint4(y0, y1, y2, m.stream) : make_uint4(x0, x1, x2, m.stream), m.key0, m.key1);
  const double u1 = ((double)r.y + 0.5) * 0x1p-32, u2 = ((double)r.z + 0.5) * 0x1p-32;
  const double n = sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
  return m.ln_mu + m.ln_sigma * n;
}

// Weight of a ph-ph channel of row l (emission: prefactor, twice for a folded
// pair; absorption: twice the prefactor) times |V3|^2 times the delta of its
// energy mismatch x: |V3|^2 delta(x) = exp(ln |V3|^2 - (x / sigma)^2) /
// (sigma sqrt(pi)), one exponential.  Positions are relative to the instance.
__device__ __forceinline__ double mf_weight(const PpModel& m, bool em, uint32_t pl, uint32_t pa, uint32_t pb,
                                            const double* __restrict__ hwi) {
  const double wl = hwi[pl], wa = hwi[pa], wb = hwi[pb];
  const uint32_t l = pl - m.n_el, a = pa - m.n_el, b = pb - m.n_el;
  const double lv = model_ln_v2(m, l, a, b);
  const double u = (em ? -wl + wa + wb : wl - wa + wb) * m.rcp_sigma;
  const double f = em ? ((m.folded && a < b) ? 2.0 : 1.0) : 2.0;
  return f * m.pre_norm * exp(lv - u * u);
}

// Packed FP64 ph-ph channels [s, e) with matrix-free weights: only the
// 8-byte words are streamed (the weight bits in them are not read); batches
// as in seg_sum_p12.  `row_rel` is the group's first row relative to the
// instance, `hwi` the instance's state energies.
template <int G, bool DERIV>
__device__ __forceinline__ void seg_sum_pp_mf(LaneAcc<G>& acc, const RowArgs& a, int64_t s, int64_t e, int lane,
                                              const double* __restrict__ z, const double* rowv, uint32_t off,
                                              const PpModel& m, uint32_t row_rel, const double* __restrict__ hwi) {
  if (s >= e) return;
  const v4u* A2 = reinterpret_cast<const v4u*>(a.pk);
  const int P = a.pack_p;
  const uint32_t pmask = (1u << P) - 1u;
  const int64_t p_end = (e + 1) / 2;
  int64_t pb = s / 2;
  v4u c[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int64_t q = pb + lane + 64 * j;
    c[j] = v4u{0u, 0u, 0u, 0u};
    if (q < p_end) c[j] = __builtin_nontemporal_load(A2 + q);
  }
  for (;;) {
    double g0[4], g1[4];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      g0[2 * j] = z[(c[j].x & pmask) + off];
      g1[2 * j] = z[(c[j].y & pmask) + off];
      g0[2 * j + 1] = z[(c[j].z & pmask) + off];
      g1[2 * j + 1] = z[(c[j].w & pmask) + off];
    }
    const int64_t nb = pb + 128;
    const bool more = nb < p_end;
    v4u n[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      n[j] = v4u{0u, 0u, 0u, 0u};
      const int64_t q = nb + lane + 64 * j;
      if (more && q < p_end) n[j] = __builtin_nontemporal_load(A2 + q);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t ca = 2 * (pb + lane + 64 * j);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (ca + h < s || ca + h >= e) continue;
        const uint32_t lo = h ? c[j].z : c[j].x, hi = h ? c[j].w : c[j].y;
        const int tag = G == 1 ? 0 : (int)((lo >> P) & 15u);
        const bool em = (hi >> P) & 1u;
        const double w = mf_weight(m, em, row_rel + (uint32_t)tag, lo & pmask, hi & pmask, hwi);
        const double xr = rowv[tag];
        acc.add(tag, term_w<K_PP, DERIV>(em, w, g0[2 * j + h], g1[2 * j + h], xr, xr + 1.0));
      }
    }
    if (!more) break;
#pragma unroll
    for (int j = 0; j < 2; ++j) c[j] = n[j];
    pb = nb;
  }
}

// One wavefront per block, so the LDS a block needs is one wavefront's
// accumulator slots and occupancy is not capped by whole 4-wave blocks.
template <int G, bool PACK, bool DERIV, bool MF = false>
__global__ __launch_bounds__(64) void k_items(RowArgs a) {
  __shared__ double acc_lds[1][G][64];
  __shared__ double rowv[1][kMaxGroupRows];
  const int wave = 0;
  const int lane = threadIdx.x & 63;
  const int64_t ii = blockIdx.x;
  bool active = ii < a.n_items;
  int64_t it = 0;
  Item item{};
  Group g{};
  if (active) {
    it = a.order[ii];
    item = a.items[it];
    g = a.groups[item.group];
    if (a.st && a.st[g.inst].done) active = false;
  }
  if (G > 1) {
#pragma unroll
    for (int j = 0; j < G; ++j) acc_lds[wave][j][lane] = 0.0;
  }
  if (active && lane < g.nrows) rowv[wave][lane] = a.z[g.row0 + lane];
  __syncthreads();
  LaneAcc<G> acc{&acc_lds[wave][0][lane], 0.0};
  if (active) {
    const double* rv = rowv[wave];
    const int64_t m = g.split;
    const int64_t lo_pe = item.lo, hi_pe = item.hi < m ? item.hi : m;
    const int64_t lo_pp = item.lo > m ? item.lo : m, hi_pp = item.hi;
    if constexpr (PACK) {
      const uint32_t off = (uint32_t)a.info[g.inst].off;
      if (!g.phonon) {
        if (a.parts & 1) seg_sum_p12<G, K_EPH, DERIV>(acc, a, item.lo, item.hi, lane, a.z, rv, off);
      } else {
        if (a.parts & 2) seg_sum_p12<G, K_PHE, DERIV>(acc, a, lo_pe, hi_pe, lane, a.z, rv, off);
        if (a.parts & 4) {
          if constexpr (MF) {
            const PpModel m = a.ppm[g.inst];
            seg_sum_pp_mf<G, DERIV>(acc, a, lo_pp, hi_pp, lane, a.z, rv, off, m, (uint32_t)g.row0 - off,
                                    a.hw + off);
          } else {
            seg_sum_p12<G, K_PP, DERIV>(acc, a, lo_pp, hi_pp, lane, a.z, rv, off);
          }
        }
      }
    } else {
      if (!g.phonon) {
        if (a.parts & 1) seg_sum<G, 64, K_EPH, DERIV>(acc, a.ch, item.lo, item.hi, lane, a.z, rv);
      } else {
        if (a.parts & 2) seg_sum<G, 64, K_PHE, DERIV>(acc, a.ch, lo_pe, hi_pe, lane, a.z, rv);
        if (a.parts & 4) seg_sum<G, 64, K_PP, DERIV>(acc, a.ch, lo_pp, hi_pp, lane, a.z, rv);
      }
    }
  }
  if (G == 1) {
    double v = acc.reg;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (active && lane == 0) a.partial[it * kMaxGroupRows] = v;
  } else {
    __syncthreads();
    if (active && lane < g.nrows) {
      // row `lane` of the group: its slot in every lane, in lane order
      const double* p = acc_lds[wave][lane];
      double s = 0.0;
      for (int l = 0; l < 64; ++l) s += p[l];
      a.partial[it * kMaxGroupRows + lane] = s;
    }
  }
}

template <bool PACK, bool DERIV, bool MF = false>
hipError_t launch_items_fmt(const RowArgs& a, int slots, hipStream_t s) {
  const int64_t nb = a.n_items;
  switch (slots) {
    case 1: hipLaunchKernelGGL((k_items<1, PACK, DERIV, MF>), dim3((unsigned)nb), dim3(64), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_items<8, PACK, DERIV, MF>), dim3((unsigned)nb), dim3(64), 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_items<16, PACK, DERIV, MF>), dim3((unsigned)nb), dim3(64), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <bool DERIV>
hipError_t launch_tiled_fmt(const RowArgs& a, int slots, hipStream_t s);

hipError_t launch_items(const RowArgs& a, int slots, hipStream_t s) {
  if (a.n_items == 0) return hipSuccess;
  if (a.pk) {
    if (!a.pkw || !a.info || a.pack_p < 1 || a.pack_p > 19 || a.pack_m != std::min(80 - 2 * a.pack_p, 52))
      return hipErrorInvalidValue;
    if (a.ppm) {   // matrix-free ph-ph weights (per-item launch only)
      if (a.blocks || !a.hw) return hipErrorInvalidValue;
      return a.deriv ? launch_items_fmt<true, true, true>(a, slots, s) : launch_items_fmt<true, false, true>(a, slots, s);
    }
    if (a.blocks) {
      if (a.n_blocks == 0) return hipSuccess;
      if (!a.border || !a.tiles || !a.bnd) return hipErrorInvalidValue;
      return a.deriv ? launch_tiled_fmt<true>(a, slots, s) : launch_tiled_fmt<false>(a, slots, s);
    }
    return a.deriv ? launch_items_fmt<true, true>(a, slots, s) : launch_items_fmt<true, false>(a, slots, s);
  }
  return a.deriv ? launch_items_fmt<false, true>(a, slots, s) : launch_items_fmt<false, false>(a, slots, s);
}

// Create time: the 16-byte FP64 channels to the packed 12-byte layout.
__global__ void k_pack12(const Channel* ch, int64_t n_ch, const Group* groups, int64_t n_groups,
                         const InstInfo* info, int P, int M, uint64_t* pk, uint32_t* pkw) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_ch) return;
  int64_t lo = 0, hi = n_groups - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (groups[mid].start <= c) lo = mid;
    else hi = mid - 1;
  }
  const Group g = groups[lo];
  const Channel x = ch[c];
  const bool live = c >= g.start && c < g.end;     // slots between instances stay zero
  const uint32_t off = (uint32_t)info[g.inst].off, pmask = (1u << P) - 1u;
  uint64_t bits = live ? (uint64_t)__double_as_longlong(x.w) & 0x7fffffffffffffffull : 0ull;
  const int sh = 52 - M;
  if (sh > 0) bits = (bits + ((1ull << (sh - 1)) - 1ull) + ((bits >> sh) & 1ull)) >> sh;   // nearest even
  const uint32_t whigh = (uint32_t)(bits >> 32);   // at most min(59 - 2P, 31) bits
  const uint32_t p0 = live ? (((uint32_t)x.i0 & (uint32_t)kPosMask) - off) & pmask : 0u;
  const uint32_t p1 = live ? ((x.i1 & (uint32_t)kPosMask) - off) & pmask : 0u;
  const uint32_t tag = live ? (((uint32_t)x.i0 >> kTagShift) & 15u) : 0u;
  const uint32_t em = live ? (x.i1 >> 31) : 0u;
  const int na = 28 - P;                             // weight bits held by the low half
  const uint32_t w_lo = p0 | (tag << P) | ((whigh & ((1u << na) - 1u)) << (P + 4));
  const uint32_t w_hi = p1 | (em << P) | ((whigh >> na) << (P + 1));
  pk[c] = ((uint64_t)w_hi << 32) | w_lo;
  // low weight words in tile-permuted order: within each 256-channel tile,
  // lane l's channels 2l, 2l + 1, 128 + 2l, 129 + 2l sit at 4l .. 4l + 3
  const int64_t r = c & 255;
  pkw[(c & ~(int64_t)255) | (((r & 127) >> 1) << 2) | ((r >> 7) << 1) | (r & 1)] = (uint32_t)bits;
}

hipError_t launch_pack12(const Channel* ch, int64_t n_ch, const Group* groups, int64_t n_groups,
                         const InstInfo* info, int p_bits, int m_bits, uint64_t* pk, uint32_t* pkw, hipStream_t s) {
  if (n_ch == 0) return hipSuccess;
  if (p_bits < 1 || p_bits > 19 || m_bits != std::min(80 - 2 * p_bits, 52)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pack12, dim3((unsigned)((n_ch + 255) / 256)), dim3(256), 0, s, ch, n_ch, groups, n_groups,
                     info, p_bits, m_bits, pk, pkw);
  return hipGetLastError();
}

// One thread per row: the row's collision integral is minus the sum of its
// group's item sums (in item order), then the plain or stage epilogue.
template <bool STAGE>
__global__ __launch_bounds__(256) void k_finish_rows(FinishArgs f) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= f.n_rows) return;
  const int32_t gi = f.row_group[row];
  const Group g = f.groups[gi];
  if (STAGE && f.st[g.inst].done) return;
  const int j = (int)(row - g.row0);
  double tot = 0.0;
  for (int64_t it = f.item_ptr[gi]; it < f.item_ptr[gi + 1]; ++it) tot += f.partial[it * kMaxGroupRows + j];
  double kv = -tot;
  if (!STAGE) {
    f.out[row] = kv;
    return;
  }
  if (f.forcing && g.phonon) kv += f.forcing[row];
  const double h = f.st[g.inst].h_use;
  const double yr = f.y[row];
  f.k[f.stage][row] = kv;
  if (!f.last) {
    double sum = 0.0;
    for (int q = 0; q < f.stage; ++q) sum += f.a[q] * f.k[q][row];
    sum += f.a[f.stage] * kv;
    f.zout[row] = yr + h * sum;
  } else {
    double sb = 0.0, sd = 0.0;
    for (int q = 0; q < f.stage; ++q) {
      const double kq = f.k[q][row];
      sb += f.b[q] * kq;
      sd += f.d[q] * kq;
    }
    sb += f.b[f.stage] * kv;
    sd += f.d[f.stage] * kv;
    f.ynew[row] = yr + h * sb;
    f.lte[row] = h * sd;
  }
}

hipError_t launch_finish_rows(const FinishArgs& f, bool stage, hipStream_t s) {
  if (f.n_rows == 0) return hipSuccess;
  const unsigned nb = (unsigned)((f.n_rows + 255) / 256);
  if (stage) hipLaunchKernelGGL(k_finish_rows<true>, dim3(nb), dim3(256), 0, s, f);
  else hipLaunchKernelGGL(k_finish_rows<false>, dim3(nb), dim3(256), 0, s, f);
  return hipGetLastError();
}

// ------------------------------------------------------------ mixed precision
#ifndef MIX_PAIRS
#define MIX_PAIRS 2
#endif
// Weights are stored relative to the FP32 scale of their 512-channel block:
// by default as a small float (6-bit exponent, min(53 - 2P, 23)-bit
// mantissa) in the same 64-bit word as the P-bit partner positions, else as
// FP16 heads extended by an 11-bit significand tail held in the index word
// (or FP16 alone, or BF16 for e-ph and ph-e, on request); the factors are
// evaluated in FP32 from one FP32 word per state (4-byte gathers):
//   phonon:   N; N + 1 is formed in FP32 (relative error <= 2u for N >= 0);
//   electron: c = f if f <= 1/2, else c = 1 - f (formed in FP64), rounded to
//             FP32 with the significand's lowest bit replaced by the choice;
//             the other factor is 1 - c in FP32.  Both f and 1 - f come back
//             within 4u relative for 0 <= f <= 1 (u = 2^-24), however close
//             f is to 0 or 1, and the code is unambiguous for any real f.
// Every lane keeps a Neumaier compensated FP32 sum per row of the group, and
// the lanes' sums and compensations are added in FP64.
__device__ __forceinline__ float bf16_to_f(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ float f16_to_f(uint32_t h) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
}

__device__ __forceinline__ float2 el_pair(float v) {   // (f, 1 - f)
  const uint32_t b = __float_as_uint(v);
  const float c = __uint_as_float(b & ~1u);            // flag cleared: f = 1 stays exact
  const float o = 1.0f - c;
  return (b & 1u) ? make_float2(o, c) : make_float2(c, o);
}
__device__ __forceinline__ float2 ph_pair(float v) { return make_float2(v, v + 1.0f); }   // (N, N + 1)

struct MixAcc {
  float2* slot;  // this lane's (sum, compensation) of row j at slot[64 * j]
  __device__ __forceinline__ void add(int tag, float x) {
    float2 a = slot[64 * tag];
    const float t = a.x + x;
    if (fabsf(a.x) >= fabsf(x)) a.y += (a.x - t) + x;
    else a.y += (x - t) + a.x;
    a.x = t;
    slot[64 * tag] = a;
  }
};

template <int KIND>
__device__ __forceinline__ float term_f(bool em, float w, float v0, float v1, float2 xr) {
  const float2 g0 = KIND == K_PP ? ph_pair(v0) : el_pair(v0);
  const float2 g1 = KIND == K_PHE ? el_pair(v1) : ph_pair(v1);
  if (KIND == K_EPH) {         // xr = (f_r, 1-f_r), g0 = (f_s, 1-f_s), g1 = (N_p, N_p+1)
    const float gain = xr.x * g0.y * (em ? g1.y : g1.x);
    const float loss = xr.y * g0.x * (em ? g1.x : g1.y);
    return w * (gain - loss);
  } else if (KIND == K_PHE) {  // xr = (N_p, N_p+1), g0 = (f_r, 1-f_r), g1 = (f_s, 1-f_s)
    const float gain = g0.x * g1.y * xr.x;
    const float loss = g0.y * g1.x * xr.y;
    return w * (gain - loss);
  } else {                     // xr = (N, N+1), g0 = (N_a, N_a+1), g1 = (N_b, N_b+1)
    const float gain = xr.x * g0.y * (em ? g1.y : g1.x);
    const float loss = xr.y * g0.x * (em ? g1.x : g1.y);
    return w * (gain - loss);
  }
}

// State position of a channel's partner word: 24 bits in the 10-byte
// formats; P bits relative to the instance's offset `off` when packed.
template <bool PACK>
__device__ __forceinline__ uint32_t mix_pos(uint32_t v, uint32_t pmask, uint32_t off) {
  return PACK ? (v & pmask) + off : v & (uint32_t)kMixPosMask;
}

// One channel of the mixed stream: decode the weight (packed small float;
// FP16 head and tail; or BF16), form w * factor in FP32 and add it to its
// row's compensated lane slot.
template <int KIND, bool PACK>
__device__ __forceinline__ void chan_mixed(MixAcc& acc, const MixArgs& a, uint32_t ix, uint32_t iy,
                                           uint32_t head, float sc, float g0, float g1, const float2* rowv) {
  int tag;
  float w;
  if constexpr (PACK) {
    const int P = a.pack_p, M = a.pack_m;
    tag = (ix >> P) & 15;
    const uint32_t wb = (ix >> (P + 4)) | (((iy & 0x7fffffffu) >> P) << (28 - P));
    const uint32_t E = wb >> M, m = wb & ((1u << M) - 1u);
    w = E ? __uint_as_float(((E + 64u) << 23) | (m << (23 - M))) : 0.0f;
  } else {
    tag = (ix >> kMixTagShift) & 15;
    if (KIND != K_PP && a.wfmt == RTBTE_W_BF16_EPH) {
      w = bf16_to_f(head);
    } else {
      // the tail fills FP32 significand bits 2..12, below the head's 10
      const uint32_t tail = (ix >> 28) | ((iy >> 20) & 0x7f0u);
      w = __uint_as_float(__float_as_uint(f16_to_f(head)) | (tail << 2));
    }
  }
  acc.add(tag, term_f<KIND>((int32_t)iy < 0, w * sc, g0, g1, rowv[tag]));
}

// Channels [s, e) of one kind.  The stream is read as channel pairs (16 B of
// words, plus 4 B of weight heads in the 10-byte formats), lanes on consecutive pairs,
// kMixPairs pairs 64 apart per lane per batch, so every load instruction
// reads whole contiguous lines.  Two-stage pipeline as in the FP64 kernel:
// the gathers of batch k are issued before the stream loads of batch k+1.
// A batch (at most 512 channels) spans at most two 512-channel scale blocks,
// whose scales are read once per batch with scalar loads.
constexpr int kMixPairs = MIX_PAIRS;
template <int KIND, bool PACK>
__device__ __forceinline__ void seg_sum_mixed(MixAcc& acc, const MixArgs& a, int64_t s, int64_t e, int lane,
                                              const float2* rowv, uint32_t off) {
  if (s >= e) return;
  constexpr int NP = kMixPairs;
  const uint32_t pmask = PACK ? (1u << a.pack_p) - 1u : 0u;
  const v4i* idx2 = reinterpret_cast<const v4i*>(a.idx);
  const uint32_t* w2 = reinterpret_cast<const uint32_t*>(a.wq);
  const int64_t p_end = (e + 1) / 2;          // pairs [s / 2, p_end)
  int64_t pb = s / 2;                          // first pair of the batch (wave-uniform)
  v4i c[NP];
  uint32_t h[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    const int64_t q = pb + lane + 64 * j;
    c[j] = v4i{0, 0, 0, 0};
    h[j] = 0;
    if (q < p_end) {
      c[j] = __builtin_nontemporal_load(idx2 + q);
      if (!PACK) h[j] = __builtin_nontemporal_load(w2 + q);
    }
  }
  for (;;) {
    float g0[2 * NP], g1[2 * NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      g0[2 * j] = a.pop[mix_pos<PACK>((uint32_t)c[j].x, pmask, off)];
      g1[2 * j] = a.pop[mix_pos<PACK>((uint32_t)c[j].y, pmask, off)];
      g0[2 * j + 1] = a.pop[mix_pos<PACK>((uint32_t)c[j].z, pmask, off)];
      g1[2 * j + 1] = a.pop[mix_pos<PACK>((uint32_t)c[j].w, pmask, off)];
    }
    const int64_t blk = __builtin_amdgcn_readfirstlane((int)(pb / (kMixBlock / 2)));
    const float s_lo = a.scale[blk];
    const float s_hi = a.scale[blk + 1 < a.n_scale ? blk + 1 : blk];
    const int64_t nb = pb + 64 * NP;
    const bool more = nb < p_end;
    v4i n[NP];
    uint32_t m[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      n[j] = v4i{0, 0, 0, 0};
      m[j] = 0;
    }
    if (more) {
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        const int64_t q = nb + lane + 64 * j;
        if (q < p_end) {
          n[j] = __builtin_nontemporal_load(idx2 + q);
          if (!PACK) m[j] = __builtin_nontemporal_load(w2 + q);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const int64_t q = pb + lane + 64 * j;
      const float sc = q / (kMixBlock / 2) == blk ? s_lo : s_hi;
      const int64_t ca = 2 * q;
      if (ca >= s && ca < e)
        chan_mixed<KIND, PACK>(acc, a, c[j].x, c[j].y, h[j] & 0xffffu, sc, g0[2 * j], g1[2 * j], rowv);
      if (ca + 1 >= s && ca + 1 < e)
        chan_mixed<KIND, PACK>(acc, a, c[j].z, c[j].w, h[j] >> 16, sc, g0[2 * j + 1], g1[2 * j + 1], rowv);
    }
    if (!more) break;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      c[j] = n[j];
      h[j] = m[j];
    }
    pb = nb;
  }
}

// Mixed precision, packed 8-byte words, ph-ph channels [s, e) with
// matrix-free weights: the weight is formed in FP64 and rounded to FP32 (no
// block scale); populations, factors and sums as in seg_sum_mixed.
__device__ __forceinline__ void seg_sum_mixed_pp_mf(MixAcc& acc, const MixArgs& a, int64_t s, int64_t e, int lane,
                                                    const float2* rowv, uint32_t off, const PpModel& m,
                                                    uint32_t row_rel, const double* __restrict__ hwi) {
  if (s >= e) return;
  constexpr int NP = kMixPairs;
  const uint32_t pmask = (1u << a.pack_p) - 1u;
  const int P = a.pack_p;
  const v4i* idx2 = reinterpret_cast<const v4i*>(a.idx);
  const int64_t p_end = (e + 1) / 2;
  int64_t pb = s / 2;
  v4i c[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    const int64_t q = pb + lane + 64 * j;
    c[j] = v4i{0, 0, 0, 0};
    if (q < p_end) c[j] = __builtin_nontemporal_load(idx2 + q);
  }
  for (;;) {
    float g0[2 * NP], g1[2 * NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      g0[2 * j] = a.pop[((uint32_t)c[j].x & pmask) + off];
      g1[2 * j] = a.pop[((uint32_t)c[j].y & pmask) + off];
      g0[2 * j + 1] = a.pop[((uint32_t)c[j].z & pmask) + off];
      g1[2 * j + 1] = a.pop[((uint32_t)c[j].w & pmask) + off];
    }
    const int64_t nb = pb + 64 * NP;
    const bool more = nb < p_end;
    v4i n[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      n[j] = v4i{0, 0, 0, 0};
      const int64_t q = nb + lane + 64 * j;
      if (more && q < p_end) n[j] = __builtin_nontemporal_load(idx2 + q);
    }
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const int64_t ca = 2 * (pb + lane + 64 * j);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (ca + h < s || ca + h >= e) continue;
        const uint32_t ix = (uint32_t)(h ? c[j].z : c[j].x), iy = (uint32_t)(h ? c[j].w : c[j].y);
        const int tag = (ix >> P) & 15;
        const bool em = (int32_t)iy < 0;
        const float w = (float)mf_weight(m, em, row_rel + (uint32_t)tag, ix & pmask, iy & pmask, hwi);
        acc.add(tag, term_f<K_PP>(em, w, g0[2 * j + h], g1[2 * j + h], rowv[tag]));
      }
    }
    if (!more) break;
#pragma unroll
    for (int j = 0; j < NP; ++j) c[j] = n[j];
    pb = nb;
  }
}

template <int G, bool PACK, bool MF = false>
__global__ __launch_bounds__(64) void k_items_mixed(MixArgs a) {
  __shared__ float2 acc_lds[G][64];
  __shared__ float2 rowv[kMaxGroupRows];
  const int lane = threadIdx.x & 63;
  const int64_t ii = blockIdx.x;
  bool active = ii < a.n_items;
  int64_t it = 0;
  Item item{};
  Group g{};
  if (active) {
    it = a.order[ii];
    item = a.items[it];
    g = a.groups[item.group];
    if (a.st && a.st[g.inst].done) active = false;
  }
#pragma unroll
  for (int j = 0; j < G; ++j) acc_lds[j][lane] = make_float2(0.f, 0.f);
  if (active && lane < g.nrows) {
    const float v = a.pop[g.row0 + lane];
    rowv[lane] = g.phonon ? ph_pair(v) : el_pair(v);
  }
  __syncthreads();
  MixAcc acc{&acc_lds[0][lane]};
  if (active) {
    const uint32_t off = PACK ? (uint32_t)a.info[g.inst].off : 0u;
    if (!g.phonon) {
      if (a.parts & 1) seg_sum_mixed<K_EPH, PACK>(acc, a, item.lo, item.hi, lane, rowv, off);
    } else {
      const int64_t m = g.split;
      if (a.parts & 2) seg_sum_mixed<K_PHE, PACK>(acc, a, item.lo, item.hi < m ? item.hi : m, lane, rowv, off);
      if (a.parts & 4) {
        if constexpr (MF) {
          const PpModel pm = a.ppm[g.inst];
          seg_sum_mixed_pp_mf(acc, a, item.lo > m ? item.lo : m, item.hi, lane, rowv, off, pm,
                              (uint32_t)g.row0 - off, a.hw + off);
        } else {
          seg_sum_mixed<K_PP, PACK>(acc, a, item.lo > m ? item.lo : m, item.hi, lane, rowv, off);
        }
      }
    }
  }
  __syncthreads();
  if (active && lane < g.nrows) {
    double sum = 0.0, comp = 0.0;
    for (int l = 0; l < 64; ++l) {
      sum += (double)acc_lds[lane][l].x;
      comp += (double)acc_lds[lane][l].y;
    }
    a.partial[it * kMaxGroupRows + lane] = sum + comp;
  }
}

template <bool PACK, bool MF = false>
hipError_t launch_items_mixed_fmt(const MixArgs& a, int slots, hipStream_t s) {
  const int64_t nb = a.n_items;
  switch (slots) {
    case 1: hipLaunchKernelGGL((k_items_mixed<1, PACK, MF>), dim3((unsigned)nb), dim3(64), 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_items_mixed<8, PACK, MF>), dim3((unsigned)nb), dim3(64), 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_items_mixed<16, PACK, MF>), dim3((unsigned)nb), dim3(64), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_tiled_mixed(const MixArgs& a, int slots, hipStream_t s);

hipError_t launch_items_mixed(const MixArgs& a, int slots, hipStream_t s) {
  if (a.n_items == 0) return hipSuccess;
  if (a.wfmt == RTBTE_W_PACK8) {
    if (!a.info || a.pack_p < 1 || a.pack_p > 20 || a.pack_m != std::min(53 - 2 * a.pack_p, 23))
      return hipErrorInvalidValue;
    if (a.ppm) {   // matrix-free ph-ph weights (per-item launch only)
      if (a.blocks || !a.hw) return hipErrorInvalidValue;
      return launch_items_mixed_fmt<true, true>(a, slots, s);
    }
    if (a.blocks) {
      if (a.n_blocks == 0) return hipSuccess;
      if (!a.border || !a.tiles || !a.bnd) return hipErrorInvalidValue;
      return launch_tiled_mixed(a, slots, s);
    }
    return launch_items_mixed_fmt<true>(a, slots, s);
  }
  return launch_items_mixed_fmt<false>(a, slots, s);
}

// One FP32 word per state, coded as described above for the mixed gathers.
__global__ void k_popf(float* pop, const double* __restrict__ z, const int32_t* row_group,
                       const Group* groups, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = z[i];
  if (groups[row_group[i]].phonon) {
    pop[i] = (float)v;
  } else {
    const bool hi = v > 0.5;
    const float c = (float)(hi ? 1.0 - v : v);
    pop[i] = __uint_as_float((__float_as_uint(c) & ~1u) | (hi ? 1u : 0u));
  }
}

hipError_t launch_popf(float* pop, const double* z, const int32_t* row_group, const Group* groups,
                       int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_popf, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pop, z, row_group, groups, n);
  return hipGetLastError();
}

// ------------------------------------------------------------- tiled launch
// (packed layouts).  A block of kTileWaves wavefronts runs one set of
// consecutive groups of one kind through a range of key blocks.  For each
// key block it stages the populations of the key block and of the window of
// other-partner positions the set's channels touch there, then each
// wavefront streams its group's channels of that key block, reading both
// partners from LDS (an other partner outside the window is gathered from
// global memory).  The row sums stay in the wavefronts' lane slots across the
// range.  The channel stream is the same as in the item kernels; a range's
// first and last batches load only the pairs inside it.

// dst[0, len) = z[start, start + len) (zero outside [0, n)), 16-byte loads
// (aligned by address) by all `nt` threads of the block.
template <typename T>
__device__ __forceinline__ void stage(T* dst, const T* __restrict__ z, int64_t start, int len, int64_t n, int tid,
                                      int nt) {
  constexpr int V = 16 / sizeof(T);
  typedef T vec __attribute__((ext_vector_type(V)));
  const int sh = (int)(((uintptr_t)(z + start) / sizeof(T)) & (V - 1));
  const int64_t g0 = start - sh;
  const int nv = (sh + len + V - 1) / V;
  for (int p = tid; p < nv; p += nt) {
    const int64_t gi = g0 + (int64_t)V * p;
    T v[V];
    if (gi >= 0 && gi + V <= n) {
      const vec w = *reinterpret_cast<const vec*>(z + gi);
#pragma unroll
      for (int k = 0; k < V; ++k) v[k] = w[k];
    } else {
#pragma unroll
      for (int k = 0; k < V; ++k) v[k] = (gi + k >= 0 && gi + k < n) ? z[gi + k] : T(0);
    }
    const int li = V * p - sh;
#pragma unroll
    for (int k = 0; k < V; ++k)
      if (li + k >= 0 && li + k < len) dst[li + k] = v[k];
  }
}

// The staged windows of one key block: key positions [klo, klo + klen),
// other-partner positions [olo, olo + olen) (olen = 0: none staged).
template <typename T>
struct Windows {
  const T* key;
  const T* oth;
  uint32_t klo, klen, olo, olen;
  // Populations of a channel whose (masked-in) partner words are lo, hi:
  // the key from LDS; the other from LDS, or from `glob` in a tile without
  // an other-partner window.
  template <int KIND>
  __device__ __forceinline__ void get(uint32_t lo, uint32_t hi, uint32_t pmask, bool valid,
                                      const T* __restrict__ glob, T& g0, T& g1) const {
    const uint32_t kp = (KIND == K_EPH ? hi : lo) & pmask;
    const uint32_t op = (KIND == K_EPH ? lo : hi) & pmask;
    const uint32_t ku = valid ? min(kp - klo, klen - 1u) : 0u;
    const T gk = key[ku];
    // olen == 0: the tile's other partners span more than the window holds
    // and are all gathered from global memory (a choice made per tile, so
    // the branch is the same for every lane)
    T go;
    if (olen) go = oth[valid ? min(op - olo, olen - 1u) : 0u];
    else go = glob[op];
    if (KIND == K_EPH) { g0 = go; g1 = gk; }
    else { g0 = gk; g1 = go; }
  }
};

// Packed FP64 channels [s, e) of one kind against staged windows: the batch
// structure of seg_sum_p12, loads restricted to the pairs of [s, e).
template <int G, int KIND, bool DERIV>
__device__ __forceinline__ void seg_sum_p12_win(LaneAcc<G>& acc, const RowArgs& a, int64_t s, int64_t e, int lane,
                                                const double* __restrict__ zi, const double* rowv,
                                                const Windows<double>& w) {
  if (s >= e) return;
  const v4u* A2 = reinterpret_cast<const v4u*>(a.pk);
  const v4u* B4 = reinterpret_cast<const v4u*>(a.pkw);
  const int P = a.pack_p, sh = 52 - a.pack_m;
  const uint32_t pmask = (1u << P) - 1u;
  const int64_t p_beg = s >> 1, p_end = (e + 1) >> 1;   // pairs [p_beg, p_end)
  int64_t pb = p_beg & ~(int64_t)127;
  v4u c0 = v4u{0u, 0u, 0u, 0u}, c1 = c0, wl = c0;
  {
    const int64_t q0 = pb + lane, q1 = q0 + 64;
    const bool in0 = q0 >= p_beg && q0 < p_end, in1 = q1 >= p_beg && q1 < p_end;
    if (in0) c0 = __builtin_nontemporal_load(A2 + q0);
    if (in1) c1 = __builtin_nontemporal_load(A2 + q1);
    if (in0 || in1) wl = __builtin_nontemporal_load(B4 + pb / 2 + lane);
  }
  for (;;) {
    const v4u c[2] = {c0, c1};
    double g0[4], g1[4];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t ca = 2 * (pb + lane + 64 * j);
      w.template get<KIND>(c[j].x, c[j].y, pmask, ca >= s && ca < e, zi, g0[2 * j], g1[2 * j]);
      w.template get<KIND>(c[j].z, c[j].w, pmask, ca + 1 >= s && ca + 1 < e, zi, g0[2 * j + 1], g1[2 * j + 1]);
    }
    const int64_t nb = pb + 128;
    const bool more = nb < p_end;
    v4u n0 = v4u{0u, 0u, 0u, 0u}, n1 = n0, m = n0;
    if (more) {   // the first pair of the next batch is inside the range
      const int64_t q0 = nb + lane, q1 = q0 + 64;
      const bool in0 = q0 < p_end, in1 = q1 < p_end;
      if (in0) n0 = __builtin_nontemporal_load(A2 + q0);
      if (in1) n1 = __builtin_nontemporal_load(A2 + q1);
      if (in0 || in1) m = __builtin_nontemporal_load(B4 + nb / 2 + lane);
    }
    const uint32_t wlo[4] = {wl.x, wl.y, wl.z, wl.w};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t ca = 2 * (pb + lane + 64 * j);
      if (ca >= s && ca < e)
        chan_p12<G, KIND, DERIV>(acc, c[j].x, c[j].y, wlo[2 * j], g0[2 * j], g1[2 * j], rowv, P, sh);
      if (ca + 1 >= s && ca + 1 < e)
        chan_p12<G, KIND, DERIV>(acc, c[j].z, c[j].w, wlo[2 * j + 1], g0[2 * j + 1], g1[2 * j + 1], rowv, P, sh);
    }
    if (!more) break;
    c0 = n0;
    c1 = n1;
    wl = m;
    pb = nb;
  }
}

template <int G, bool DERIV>
__global__ __launch_bounds__(64 * kTileWaves) void k_items_tiled(RowArgs a) {
  __shared__ double kwin[kTileKey64];
  __shared__ double owin[kTileOther64];
  __shared__ double acc_lds[kTileWaves][G][64];
  __shared__ double rowv[kTileWaves][kMaxGroupRows];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if ((int64_t)blockIdx.x >= a.n_blocks) return;
  const TileBlock* bp = a.blocks + a.border[blockIdx.x];
  const TileBlock b = *bp;
  if (a.st && a.st[b.inst].done) return;            // the whole block
  const InstInfo inf = a.info[b.inst];
  const uint32_t n_inst = (uint32_t)(inf.n_el + inf.n_ph);
  const double* zi = a.z + inf.off;
  const int it = bp->item[wave];                    // per-wave fields read by address
  const int64_t bo = bp->bndo[wave];
  Group g{};
  if (it >= 0) g = a.groups[a.items[it].group];
#pragma unroll
  for (int j = 0; j < G; ++j) acc_lds[wave][j][lane] = 0.0;
  if (it >= 0 && lane < g.nrows) rowv[wave][lane] = a.z[g.row0 + lane];
  LaneAcc<G> acc{&acc_lds[wave][0][lane], 0.0};
  if ((a.parts >> b.kind) & 1) {
    for (int j = b.j0; j < b.j1; ++j) {
      const Tile t = a.tiles[b.tile0 + (j - b.j0)];
      if (t.lo == kTileEmpty) continue;              // the same for the whole block
      const uint32_t klo = (uint32_t)j * kTileKey64;
      const uint32_t klen = min((uint32_t)kTileKey64, n_inst - klo);
      __syncthreads();                               // the previous key block's reads are done
      stage(kwin, a.z, inf.off + klo, (int)klen, a.ny, tid, 64 * kTileWaves);
      stage(owin, a.z, inf.off + t.lo, (int)t.len, a.ny, tid, 64 * kTileWaves);
      __syncthreads();
      if (it >= 0) {
        const int64_t s = a.bnd[bo + j], e = a.bnd[bo + j + 1];
        const Windows<double> w{kwin, owin, klo, klen, t.lo, t.len};
        if (b.kind == K_EPH) seg_sum_p12_win<G, K_EPH, DERIV>(acc, a, s, e, lane, zi, rowv[wave], w);
        else if (b.kind == K_PHE) seg_sum_p12_win<G, K_PHE, DERIV>(acc, a, s, e, lane, zi, rowv[wave], w);
        else seg_sum_p12_win<G, K_PP, DERIV>(acc, a, s, e, lane, zi, rowv[wave], w);
      }
    }
  }
  __syncthreads();
  if (it < 0) return;
  if (G == 1) {              // one-row groups accumulate in a register
    double v = acc.reg;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) a.partial[(int64_t)it * kMaxGroupRows] = v;
  } else if (lane < g.nrows) {
    // row `lane` of the group: its slot in every lane, in lane order
    const double* p = acc_lds[wave][lane];
    double sum = 0.0;
    for (int l = 0; l < 64; ++l) sum += p[l];
    a.partial[(int64_t)it * kMaxGroupRows + lane] = sum;
  }
}

template <bool DERIV>
hipError_t launch_tiled_fmt(const RowArgs& a, int slots, hipStream_t s) {
  const dim3 grid((unsigned)a.n_blocks), blk(64 * kTileWaves);
  switch (slots) {
    case 1: hipLaunchKernelGGL((k_items_tiled<1, DERIV>), grid, blk, 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_items_tiled<8, DERIV>), grid, blk, 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_items_tiled<16, DERIV>), grid, blk, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Mixed precision (packed 8-byte words) against staged windows of 4-byte
// population codes: the batch structure of seg_sum_mixed.
template <int KIND>
__device__ __forceinline__ void seg_sum_mixed_win(MixAcc& acc, const MixArgs& a, int64_t s, int64_t e, int lane,
                                                  const float2* rowv, const float* __restrict__ popi,
                                                  const Windows<float>& w) {
  if (s >= e) return;
  constexpr int NP = kMixPairs;
  const uint32_t pmask = (1u << a.pack_p) - 1u;
  const v4i* idx2 = reinterpret_cast<const v4i*>(a.idx);
  const int64_t p_beg = s >> 1, p_end = (e + 1) >> 1;
  int64_t pb = p_beg;
  v4i c[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    const int64_t q = pb + lane + 64 * j;
    c[j] = v4i{0, 0, 0, 0};
    if (q < p_end) c[j] = __builtin_nontemporal_load(idx2 + q);
  }
  for (;;) {
    float g0[2 * NP], g1[2 * NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const int64_t ca = 2 * (pb + lane + 64 * j);
      w.template get<KIND>((uint32_t)c[j].x, (uint32_t)c[j].y, pmask, ca >= s && ca < e, popi, g0[2 * j],
                           g1[2 * j]);
      w.template get<KIND>((uint32_t)c[j].z, (uint32_t)c[j].w, pmask, ca + 1 >= s && ca + 1 < e, popi,
                           g0[2 * j + 1], g1[2 * j + 1]);
    }
    const int64_t blk = __builtin_amdgcn_readfirstlane((int)(pb / (kMixBlock / 2)));
    const float s_lo = a.scale[blk];
    const float s_hi = a.scale[blk + 1 < a.n_scale ? blk + 1 : blk];
    const int64_t nb = pb + 64 * NP;
    const bool more = nb < p_end;
    v4i n[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) n[j] = v4i{0, 0, 0, 0};
    if (more) {
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        const int64_t q = nb + lane + 64 * j;
        if (q < p_end) n[j] = __builtin_nontemporal_load(idx2 + q);
      }
    }
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const int64_t q = pb + lane + 64 * j;
      const float sc = q / (kMixBlock / 2) == blk ? s_lo : s_hi;
      const int64_t ca = 2 * q;
      if (ca >= s && ca < e)
        chan_mixed<KIND, true>(acc, a, (uint32_t)c[j].x, (uint32_t)c[j].y, 0u, sc, g0[2 * j], g1[2 * j], rowv);
      if (ca + 1 >= s && ca + 1 < e)
        chan_mixed<KIND, true>(acc, a, (uint32_t)c[j].z, (uint32_t)c[j].w, 0u, sc, g0[2 * j + 1], g1[2 * j + 1],
                               rowv);
    }
    if (!more) break;
#pragma unroll
    for (int j = 0; j < NP; ++j) c[j] = n[j];
    pb = nb;
  }
}

template <int G>
__global__ __launch_bounds__(64 * kTileWaves) void k_items_mixed_tiled(MixArgs a) {
  __shared__ float kwin[kTileKey32];
  __shared__ float owin[kTileOther32];
  __shared__ float2 acc_lds[kTileWaves][G][64];
  __shared__ float2 rowv[kTileWaves][kMaxGroupRows];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if ((int64_t)blockIdx.x >= a.n_blocks) return;
  const TileBlock* bp = a.blocks + a.border[blockIdx.x];
  const TileBlock b = *bp;
  if (a.st && a.st[b.inst].done) return;
  const InstInfo inf = a.info[b.inst];
  const uint32_t n_inst = (uint32_t)(inf.n_el + inf.n_ph);
  const float* popi = a.pop + inf.off;
  const int it = bp->item[wave];
  const int64_t bo = bp->bndo[wave];
  Group g{};
  if (it >= 0) g = a.groups[a.items[it].group];
#pragma unroll
  for (int j = 0; j < G; ++j) acc_lds[wave][j][lane] = make_float2(0.f, 0.f);
  if (it >= 0 && lane < g.nrows) {
    const float v = a.pop[g.row0 + lane];
    rowv[wave][lane] = g.phonon ? ph_pair(v) : el_pair(v);
  }
  MixAcc acc{&acc_lds[wave][0][lane]};
  if ((a.parts >> b.kind) & 1) {
    for (int j = b.j0; j < b.j1; ++j) {
      const Tile t = a.tiles[b.tile0 + (j - b.j0)];
      if (t.lo == kTileEmpty) continue;
      const uint32_t klo = (uint32_t)j * kTileKey32;
      const uint32_t klen = min((uint32_t)kTileKey32, n_inst - klo);
      __syncthreads();
      stage(kwin, a.pop, inf.off + klo, (int)klen, a.ny, tid, 64 * kTileWaves);
      stage(owin, a.pop, inf.off + t.lo, (int)t.len, a.ny, tid, 64 * kTileWaves);
      __syncthreads();
      if (it >= 0) {
        const int64_t s = a.bnd[bo + j], e = a.bnd[bo + j + 1];
        const Windows<float> w{kwin, owin, klo, klen, t.lo, t.len};
        if (b.kind == K_EPH) seg_sum_mixed_win<K_EPH>(acc, a, s, e, lane, rowv[wave], popi, w);
        else if (b.kind == K_PHE) seg_sum_mixed_win<K_PHE>(acc, a, s, e, lane, rowv[wave], popi, w);
        else seg_sum_mixed_win<K_PP>(acc, a, s, e, lane, rowv[wave], popi, w);
      }
    }
  }
  __syncthreads();
  if (it >= 0 && lane < g.nrows) {
    double sum = 0.0, comp = 0.0;
    for (int l = 0; l < 64; ++l) {
      sum += (double)acc_lds[wave][lane][l].x;
      comp += (double)acc_lds[wave][lane][l].y;
    }
    a.partial[(int64_t)it * kMaxGroupRows + lane] = sum + comp;
  }
}

hipError_t launch_tiled_mixed(const MixArgs& a, int slots, hipStream_t s) {
  const dim3 grid((unsigned)a.n_blocks), blk(64 * kTileWaves);
  switch (slots) {
    case 1: hipLaunchKernelGGL((k_items_mixed_tiled<1>), grid, blk, 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_items_mixed_tiled<8>), grid, blk, 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_items_mixed_tiled<16>), grid, blk, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Create time: first channel of each key block of each segment (binary
// search over the segment's channels, sorted by key).
__global__ void k_key_bounds(const uint64_t* words, int P, const SegRange* segs, int64_t n_segs, int64_t key_len,
                             int64_t* bnd) {
  const int64_t si = blockIdx.y * (int64_t)gridDim.x + blockIdx.x;
  if (si >= n_segs) return;
  const SegRange sg = segs[si];
  const uint32_t pmask = (1u << P) - 1u;
  for (int j = threadIdx.x; j <= sg.n_kb; j += blockDim.x) {
    const uint64_t target = (uint64_t)j * (uint64_t)key_len;
    int64_t lo = sg.lo, hi = sg.hi;   // first channel in [lo, hi) with key >= target
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      const uint64_t wd = words[mid];
      const uint32_t key = (uint32_t)(sg.kind == 0 ? (wd >> 32) : wd) & pmask;
      if (key < target) lo = mid + 1;
      else hi = mid;
    }
    bnd[sg.off + j] = lo;
  }
}

hipError_t launch_key_bounds(const uint64_t* words, int pack_p, const SegRange* segs, int64_t n_segs,
                             int64_t key_len, int64_t* bnd, hipStream_t s) {
  if (n_segs == 0) return hipSuccess;
  const int64_t gx = std::min<int64_t>(n_segs, 65535), gy = (n_segs + gx - 1) / gx;
  hipLaunchKernelGGL(k_key_bounds, dim3((unsigned)gx, (unsigned)gy), dim3(128), 0, s, words, pack_p, segs, n_segs,
                     key_len, bnd);
  return hipGetLastError();
}

// Create time: smallest and largest other-partner position of the channels
// of one key block of a set of segments, one wavefront per job.
__global__ __launch_bounds__(64) void k_tile_span(const uint64_t* words, int P, const SpanJob* jobs,
                                                  int64_t n_jobs, const int64_t* bnd, uint32_t* span) {
  const int64_t ji = blockIdx.y * (int64_t)gridDim.x + blockIdx.x;
  if (ji >= n_jobs) return;
  const SpanJob jb = jobs[ji];
  const uint32_t pmask = (1u << P) - 1u;
  uint32_t mn = 0xffffffffu, mx = 0u;
  for (int w = 0; w < kTileWaves; ++w) {
    if (jb.bndo[w] < 0) continue;
    const int64_t s = bnd[jb.bndo[w] + jb.j], e = bnd[jb.bndo[w] + jb.j + 1];
    for (int64_t c = s + threadIdx.x; c < e; c += 64) {
      const uint64_t wd = words[c];
      const uint32_t o = (uint32_t)(jb.kind == 0 ? wd : (wd >> 32)) & pmask;
      mn = min(mn, o);
      mx = max(mx, o);
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    mn = min(mn, (uint32_t)__shfl_xor((int)mn, o, 64));
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
  }
  if (threadIdx.x == 0) {
    span[2 * ji] = mn;
    span[2 * ji + 1] = mx;
  }
}

hipError_t launch_tile_span(const uint64_t* words, int pack_p, const SpanJob* jobs, int64_t n_jobs,
                            const int64_t* bnd, uint32_t* span, hipStream_t s) {
  if (n_jobs == 0) return hipSuccess;
  const int64_t gx = std::min<int64_t>(n_jobs, 65535), gy = (n_jobs + gx - 1) / gx;
  hipLaunchKernelGGL(k_tile_span, dim3((unsigned)gx, (unsigned)gy), dim3(64), 0, s, words, pack_p, jobs, n_jobs,
                     bnd, span);
  return hipGetLastError();
}

// Scale of each 512-channel block: its largest weight (rounded up to FP32)
// times `headroom` (a power of two; `headroom` alone if all are 0).  The
// 16-bit formats use 2^-15, so stored values lie in [0, 2^15] and FP16 values
// of small weights stay out of FP16's subnormal range down to 2^-29 of the
// block's largest weight; the packed 8-byte format uses 1 (values in [0, 1]).
__global__ __launch_bounds__(256) void k_mix_scales(const Channel* ch, int64_t n_ch, float headroom,
                                                    float* scale) {
  __shared__ double red[4];
  const int64_t b = blockIdx.x;
  double m = 0.0;
  for (int64_t c = b * kMixBlock + threadIdx.x; c < (b + 1) * kMixBlock && c < n_ch; c += 256)
    m = fmax(m, fabs(ch[c].w));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    // round the scale up so every scaled weight is <= 1 / headroom
    float sf = (float)m;
    if ((double)sf < m) sf = nextafterf(sf, INFINITY);
    scale[b] = (m > 0.0 ? sf : 1.0f) * headroom;
  }
}

hipError_t launch_mix_scales(const Channel* ch, int64_t n_ch, float headroom, float* scale, hipStream_t s) {
  const int64_t nb = (n_ch + kMixBlock - 1) / kMixBlock;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mix_scales, dim3((unsigned)nb), dim3(256), 0, s, ch, n_ch, headroom, scale);
  return hipGetLastError();
}

__device__ __forceinline__ uint16_t to_bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// r in [0, 2^15] (finite) to an FP16 head and an 11-bit tail: r rounded once,
// to nearest even, to 22 significant bits.  Values below FP16's normal range
// (2^-14) are plain FP16 (their tail is zero).
__device__ __forceinline__ void to_f16x(double r, uint16_t* head, uint32_t* tail) {
  const double m = fabs(r);
  if (!(m >= 0x1p-14)) {
    *head = __builtin_bit_cast(uint16_t, (_Float16)(float)r);
    *tail = 0;
    return;
  }
  int e = ilogb(m);                           // 2^e <= m < 2^(e+1)
  double q = rint(ldexp(m, 21 - e));          // in [2^21, 2^22]
  if (q >= 0x1p22) { q = 0x1p21; ++e; }
  const uint32_t sig = (uint32_t)q;           // 22 bits, leading one at bit 21
  const uint32_t sign = r < 0 ? 0x8000u : 0u;
  *head = (uint16_t)(sign | ((uint32_t)(e + 15) << 10) | ((sig >> 11) & 0x3ffu));
  *tail = sig & 0x7ffu;
}

__global__ void k_mix_convert(const Channel* ch, int64_t n_ch, const Group* groups, int64_t n_groups,
                              const float* scale, int wfmt, int2* idx, uint16_t* wq) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_ch) return;
  // the group holding channel c: last group with start <= c
  int64_t lo = 0, hi = n_groups - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (groups[mid].start <= c) lo = mid;
    else hi = mid - 1;
  }
  const Group g = groups[lo];
  const bool pp = g.phonon && c >= g.split;
  const Channel x = ch[c];
  const double r = x.w / (double)scale[c / kMixBlock];
  uint32_t tail = 0;
  if (!pp && wfmt == RTBTE_W_BF16_EPH) wq[c] = to_bf16_rne((float)r);
  else if (wfmt == RTBTE_W_F16) wq[c] = __builtin_bit_cast(uint16_t, (_Float16)(float)r);
  else to_f16x(r, &wq[c], &tail);
  const uint32_t pos0 = (uint32_t)x.i0 & (uint32_t)kPosMask, pos1 = x.i1 & (uint32_t)kPosMask;
  const uint32_t tag = ((uint32_t)x.i0 >> kTagShift) & 15u;
  const uint32_t wx = pos0 | (tag << kMixTagShift) | ((tail & 15u) << 28);
  const uint32_t wy = pos1 | ((tail >> 4) << 24) | (x.i1 & kEmBit);
  idx[c] = make_int2((int)wx, (int)wy);
}

hipError_t launch_mix_convert(const Channel* ch, int64_t n_ch, const Group* groups, int64_t n_groups,
                              const float* scale, int wfmt, int2* idx, uint16_t* wq, hipStream_t s) {
  if (n_ch == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mix_convert, dim3((unsigned)((n_ch + 255) / 256)), dim3(256), 0, s, ch, n_ch, groups,
                     n_groups, scale, wfmt, idx, wq);
  return hipGetLastError();
}

// Packed 8-byte channels: weight r = w / scale in [0, 1] as a small float,
// 6 exponent bits e (r = 2^(e - 63) (1 + m 2^-M), e >= 1; e = 0: zero, for
// r < 2^-62) over M mantissa bits, rounded once to nearest even.
__device__ __forceinline__ uint32_t to_pack_weight(double r, int M) {
  if (!(r >= 0x1p-62)) return 0u;
  const int e = ilogb(r);                                   // -62 .. 0
  const double q = rint(ldexp(r, M - e)) - ldexp(1.0, M);   // 0 .. 2^M
  uint32_t m = (uint32_t)q, E = (uint32_t)(e + 63);
  if (m >= (1u << M)) { m = 0u; E += 1u; }
  return (E << M) | m;
}

__global__ void k_mix_pack8(const Channel* ch, int64_t n_ch, const Group* groups, int64_t n_groups,
                            const InstInfo* info, const float* scale, int P, int M, int2* words) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_ch) return;
  int64_t lo = 0, hi = n_groups - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (groups[mid].start <= c) lo = mid;
    else hi = mid - 1;
  }
  const Group g = groups[lo];
  const Channel x = ch[c];
  const uint32_t off = (uint32_t)info[g.inst].off;
  const uint32_t pmask = (1u << P) - 1u;
  // slots between instances (weight 0, positions 0) hold zero words
  const bool live = c >= g.start && c < g.end;
  const uint32_t p0 = live ? (((uint32_t)x.i0 & (uint32_t)kPosMask) - off) & pmask : 0u;
  const uint32_t p1 = live ? ((x.i1 & (uint32_t)kPosMask) - off) & pmask : 0u;
  const uint32_t tag = live ? ((uint32_t)x.i0 >> kTagShift) & 15u : 0u;
  const uint32_t w = live ? to_pack_weight(x.w / (double)scale[c / kMixBlock], M) : 0u;
  const int lo_bits = 28 - P;                               // weight bits held by the first word
  const uint32_t wx = p0 | (tag << P) | ((w & ((1u << lo_bits) - 1u)) << (P + 4));
  const uint32_t wy = p1 | ((w >> lo_bits) << P) | (live ? (x.i1 & kEmBit) : 0u);
  words[c] = make_int2((int)wx, (int)wy);
}

hipError_t launch_mix_pack8(const Channel* ch, int64_t n_ch, const Group* groups, int64_t n_groups,
                            const InstInfo* info, const float* scale, int p_bits, int m_bits, int2* words,
                            hipStream_t s) {
  if (n_ch == 0) return hipSuccess;
  if (p_bits < 1 || p_bits > 20 || m_bits != std::min(53 - 2 * p_bits, 23)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mix_pack8, dim3((unsigned)((n_ch + 255) / 256)), dim3(256), 0, s, ch, n_ch, groups,
                     n_groups, info, scale, p_bits, m_bits, words);
  return hipGetLastError();
}

// ------------------------------------------------------------------ WRMS norm
// Partial sums of (v_i w_i)^2, w_i = 1/(rtol |y_i| + atol_i) (Eq. (wrms_norm),
// Eq. (wrms_weights)); grid (nchunk, n_inst), fixed summation order.
__global__ __launch_bounds__(256) void k_wrms(const double* __restrict__ v, const double* __restrict__ y,
                                              const InstInfo* info, const InstState* st,
                                              double* partial, int nchunk, Ctl c) {
  __shared__ double red[4];
  const int inst = blockIdx.y;
  if (st && st[inst].done) return;
  const InstInfo in = info[inst];
  const int64_t n = (int64_t)in.n_el + in.n_ph;
  const int64_t cs = (n + nchunk - 1) / nchunk;
  const int64_t lo = (int64_t)blockIdx.x * cs;
  const int64_t hi = lo + cs < n ? lo + cs : n;
  double acc = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
    const double atol = i < in.n_el ? c.atol_el : c.atol_ph;
    const double q = v[in.off + i] / (c.rtol * fabs(y[in.off + i]) + atol);
    acc += q * q;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[(int64_t)inst * nchunk + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

hipError_t launch_wrms(const double* v, const double* y, const InstInfo* info, const InstState* st,
                       double* partial, int n_inst, int nchunk, Ctl c, hipStream_t s) {
  hipLaunchKernelGGL(k_wrms, dim3(nchunk, n_inst), dim3(256), 0, s, v, y, info, st, partial, nchunk, c);
  return hipGetLastError();
}

__device__ __forceinline__ double wrms_total(const double* partial, int inst, int nchunk, int64_t n) {
  double s = 0.0;
  for (int j = 0; j < nchunk; ++j) s += partial[(int64_t)inst * nchunk + j];
  return sqrt(s / (double)n);
}

// ------------------------------------------------------------- step control
// PID ratio of Eq. (pid_controller) with the safeguards of the options;
// `fails` counts the consecutive failures, this one included.
__device__ double pid_eta(double eps, double e1, double e2, bool accepted, bool first, const Ctl& c,
                          int fails = 1) {
  const double e0 = fmax(eps, c.eps_floor);
  const double s2 = c.alt_sign ? 1.0 : -1.0;
  double eta = c.safety * pow(e0, -c.k1 / c.order) * pow(fmax(e1, c.eps_floor), s2 * c.k2 / c.order) *
               pow(fmax(e2, c.eps_floor), -c.k3 / c.order);
  if (accepted) return fmin(eta, first ? c.eta_max_first : c.eta_max);
  eta = fmin(fmax(eta, c.eta_fail_min), c.eta_fail_max);
  return fails >= c.small_nef ? fmin(eta, c.eta_fail_repeat) : eta;
}

__device__ void plan_next(InstState& s) {
  if (s.done) return;
  const double hc = s.h_cap > 0.0 ? fmin(s.h, s.h_cap) : s.h;
  const bool last = s.t + hc >= s.t_out;
  s.last = last;
  s.h_use = last ? s.t_out - s.t : hc;
}

__global__ void k_control(InstState* st, const double* partial, const InstInfo* info, int n_inst,
                          int nchunk, Ctl c) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= n_inst) return;
  InstState s = st[inst];
  if (s.done) return;
  s.n_attempt++;
  s.n_evals += c.stages;
  if (c.fixed) {
    // the partial sums hold the candidate state's RMS: a non-finite value
    // (the state diverged or overflowed) ends the run at the last state
    if (!isfinite(wrms_total(partial, inst, nchunk, (int64_t)info[inst].n_el + info[inst].n_ph))) {
      s.status = -5;  // RTBTE_E_NONFINITE
      s.done = 1;
      s.accepted = 0;
      st[inst] = s;
      return;
    }
    s.accepted = 1;
    s.n_accept++;
    s.steps_left--;
    s.t = s.steps_left <= 0 ? s.t_out : s.t + s.h_use;
    if (s.steps_left <= 0) s.done = 1;
    if (!s.done) { s.h_use = s.h; s.last = s.steps_left == 1; }
    st[inst] = s;
    return;
  }
  const int64_t n = (int64_t)info[inst].n_el + info[inst].n_ph;
  const double eps = wrms_total(partial, inst, nchunk, n);
  s.eps = eps;
  if (!isfinite(eps)) {
    s.status = -5;  // RTBTE_E_NONFINITE
    s.done = 1;
    s.accepted = 0;
    st[inst] = s;
    return;
  }
  if (!(s.t + s.h_use > s.t)) {  // the step no longer advances time
    s.status = -4;                // RTBTE_E_STEP
    s.done = 1;
    s.accepted = 0;
    st[inst] = s;
    return;
  }
  if (eps <= 1.0) {
    s.accepted = 1;
    const double hu = s.h_use;
    s.h = hu * pid_eta(eps, s.e1, s.e2, true, s.first != 0, c);
    s.e2 = s.e1;
    s.e1 = fmax(eps, c.eps_floor);
    s.first = 0;
    s.fails = 0;
    s.t = s.last ? s.t_out : s.t + hu;
    s.n_accept++;
    s.h_min = fmin(s.h_min, hu);
    s.h_max = fmax(s.h_max, hu);
    if (s.t >= s.t_out || s.one_step) s.done = 1;
  } else {
    s.accepted = 0;
    s.fails++;
    s.h = s.h_use * pid_eta(eps, s.e1, s.e2, false, s.first != 0, c, s.fails);
    s.n_reject++;
    if (s.fails > c.max_fails) {
      s.status = -4;  // RTBTE_E_STEP
      s.done = 1;
    }
  }
  plan_next(s);
  st[inst] = s;
}

hipError_t launch_control(InstState* st, const double* partial, const InstInfo* info, int n_inst,
                          int nchunk, Ctl c, hipStream_t s) {
  hipLaunchKernelGGL(k_control, dim3((n_inst + 63) / 64), dim3(64), 0, s, st, partial, info, n_inst,
                     nchunk, c);
  return hipGetLastError();
}

__global__ void k_commit(double* __restrict__ y, const double* __restrict__ ynew,
                         const int32_t* row_inst, const InstState* st, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int inst = row_inst ? row_inst[i] : 0;
  if (st[inst].accepted) y[i] = ynew[i];
}

__global__ __launch_bounds__(256) void k_health(const double* __restrict__ y, const InstInfo* info,
                                                int32_t* health, double tol) {
  const InstInfo in = info[blockIdx.x];
  int f_bad = 0, n_bad = 0;
  for (int64_t i = threadIdx.x; i < in.n_el; i += 256) {
    const double f = y[in.off + i];
    f_bad |= !(f >= -tol && f <= 1.0 + tol);
  }
  for (int64_t i = threadIdx.x; i < in.n_ph; i += 256) n_bad |= !(y[in.off + in.n_el + i] >= -tol);
  f_bad = __syncthreads_or(f_bad);
  n_bad = __syncthreads_or(n_bad);
  if (threadIdx.x == 0 && (f_bad || n_bad)) health[blockIdx.x] |= (f_bad ? 1 : 0) | (n_bad ? 2 : 0);
}

hipError_t launch_health(const double* y, const InstInfo* info, int32_t* health, int n_inst, double tol,
                         hipStream_t s) {
  if (n_inst == 0) return hipSuccess;
  hipLaunchKernelGGL(k_health, dim3((unsigned)n_inst), dim3(256), 0, s, y, info, health, tol);
  return hipGetLastError();
}

hipError_t launch_commit(double* y, const double* ynew, const int32_t* row_inst,
                         const InstState* st, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_commit, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, ynew, row_inst, st, n);
  return hipGetLastError();
}

// Start of a stepping call: time, target, first step size of every instance.
__global__ void k_begin(InstState* st, const double* t_in, const double* h_in, int n_inst, double t_out,
                        int one_step, double h_cap, int64_t fixed_steps, double fixed_h) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= n_inst) return;
  InstState s = st[inst];
  s.t = t_in[inst];
  s.t_start = s.t;
  s.done = 0;
  s.status = 0;
  s.accepted = 0;
  s.fails = 0;
  s.one_step = one_step;
  s.h_cap = h_cap;
  s.need_h0 = 0;
  if (fixed_steps > 0) {
    s.steps_left = fixed_steps;
    s.h = fixed_h;
    s.h_use = fixed_h;
    s.t_out = s.t + (double)fixed_steps * fixed_h;
    s.last = fixed_steps == 1;
  } else {
    s.t_out = t_out;
    if (!(s.t < s.t_out)) s.done = 1;
    if (h_in) {
      // h <= 0 asks for the starting-step estimate; an instance already at
      // or past t_out keeps the h it was given (written back unchanged)
      if (h_in[inst] > 0.0 || s.done) s.h = h_in[inst];
      else s.need_h0 = 1;
    }
    if (!s.need_h0) plan_next(s);
  }
  st[inst] = s;
}

hipError_t launch_begin(InstState* st, const double* t_in, const double* h_in, int n_inst,
                        double t_out, int one_step, double h_cap, int64_t fixed_steps,
                        double fixed_h, hipStream_t s) {
  hipLaunchKernelGGL(k_begin, dim3((n_inst + 63) / 64), dim3(64), 0, s, st, t_in, h_in, n_inst, t_out,
                     one_step, h_cap, fixed_steps, fixed_h);
  return hipGetLastError();
}

// Write t, h back and summarise: summary[0] = all done, summary[1] = worst status.
__global__ void k_finish(const InstState* st, double* t_out_buf, double* h_out_buf, int n_inst,
                         int32_t* summary) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int all = 1, worst = 0;
  for (int i = 0; i < n_inst; ++i) {
    all &= st[i].done;
    if (st[i].status < worst) worst = st[i].status;
    if (t_out_buf) t_out_buf[i] = st[i].t;
    if (h_out_buf) h_out_buf[i] = st[i].h;
  }
  summary[0] = all;
  summary[1] = worst;
}

hipError_t launch_finish(const InstState* st, double* t_out_buf, double* h_out_buf, int n_inst,
                         int32_t* summary, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, st, t_out_buf, h_out_buf, n_inst, summary);
  return hipGetLastError();
}

// -------------------------------------------------------- starting step size
// Hairer, Norsett & Wanner (Solving ODEs I, II.4), in the WRMS norm:
// d0 = ||y0||, d1 = ||f0||, h0 = 0.01 d0/d1 (1e-6 if either < 1e-5);
// d2 = ||f(y0 + h0 f0) - f0|| / h0; h1 = (0.01/max(d1,d2))^(1/(p+1));
// h = min(100 h0, h1).
__global__ void k_h0_stage1(InstState* st, const double* py, const double* pf, const InstInfo* info,
                            int n_inst, int nchunk) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= n_inst) return;
  InstState s = st[inst];
  if (!s.need_h0) return;
  const int64_t n = (int64_t)info[inst].n_el + info[inst].n_ph;
  const double d0 = wrms_total(py, inst, nchunk, n), d1 = wrms_total(pf, inst, nchunk, n);
  s.h0_d0 = d0;
  s.h0_d1 = d1;
  s.h = (d0 >= 1e-5 && d1 >= 1e-5) ? 0.01 * d0 / d1 : 1e-6;
  st[inst] = s;
}

hipError_t launch_h0_stage1(InstState* st, const double* partial_y, const double* partial_f,
                            const InstInfo* info, int n_inst, int nchunk, hipStream_t s) {
  hipLaunchKernelGGL(k_h0_stage1, dim3((n_inst + 63) / 64), dim3(64), 0, s, st, partial_y, partial_f,
                     info, n_inst, nchunk);
  return hipGetLastError();
}

__global__ void k_h0_axpy(double* out, const double* y, const double* f, const int32_t* row_inst,
                          const InstState* st, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int inst = row_inst ? row_inst[i] : 0;
  out[i] = y[i] + st[inst].h * f[i];
}

hipError_t launch_h0_axpy(double* out, const double* y, const double* f, const int32_t* row_inst,
                          const InstState* st, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_h0_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, y, f, row_inst, st, n);
  return hipGetLastError();
}

__global__ void k_sub(double* out, const double* a, const double* b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] - b[i];
}

hipError_t launch_sub(double* out, const double* a, const double* b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_sub, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, a, b, n);
  return hipGetLastError();
}

__global__ void k_h0_stage2(InstState* st, const double* pd, const InstInfo* info, int n_inst, int nchunk,
                            double order) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= n_inst) return;
  InstState s = st[inst];
  if (!s.need_h0) return;
  const int64_t n = (int64_t)info[inst].n_el + info[inst].n_ph;
  const double h0 = s.h;
  const double d2 = wrms_total(pd, inst, nchunk, n) / h0;
  const double m = fmax(s.h0_d1, d2);
  const double h1 = m > 1e-15 ? pow(0.01 / m, 1.0 / (order + 1.0)) : fmax(1e-6, h0 * 1e-3);
  s.h = fmin(100.0 * h0, h1);
  s.need_h0 = 0;
  plan_next(s);
  st[inst] = s;
}

hipError_t launch_h0_stage2(InstState* st, const double* partial_d, const InstInfo* info, int n_inst,
                            int nchunk, double order, hipStream_t s) {
  hipLaunchKernelGGL(k_h0_stage2, dim3((n_inst + 63) / 64), dim3(64), 0, s, st, partial_d, info, n_inst,
                     nchunk, order);
  return hipGetLastError();
}

// out[off + i] = sum_j coef[j] * vecs[j][off + i], i < n (MIS forcing).
struct LinComb { const double* v[4]; double c[4]; };
__global__ void k_lincomb(double* out, LinComb lc, int nv, int64_t off, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < nv; ++j) s += lc.c[j] * lc.v[j][off + i];
  out[off + i] = s;
}

hipError_t launch_lincomb(double* out, const double* const* vecs, const double* coef, int nv,
                          int64_t off, int64_t n, hipStream_t s) {
  if (nv > 4) return hipErrorInvalidValue;
  LinComb lc{};
  for (int j = 0; j < nv; ++j) { lc.v[j] = vecs[j]; lc.c[j] = coef[j]; }
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lincomb, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, lc, nv, off, n);
  return hipGetLastError();
}

// ------------------------------------------------ create-time channel preparation
// One wavefront per destination group walks the group's raw entries in their
// merged visiting order, decides which channels are kept (energy mismatch
// within the truncation, no phonon below the cutoff), and either counts them
// or writes them, tagged with their row in the group, with their weights
// prefactor * |M|^2 * delta(mismatch).  Positions come from ballots, so the
// output order is the visiting order (emission before absorption for one
// entry).
struct Kept { bool em, ab; double wem, wab; int32_t o0; uint32_t o1; };

// Destination row (instance-local) of a raw entry in the list being prepared.
__device__ __forceinline__ int32_t dest_of(const PrepArgs& p, int64_t e) {
  return p.kind == 1 ? p.i1[e] : p.row[e];
}

__device__ __forceinline__ Kept classify(const PrepArgs& p, int64_t j) {
  Kept k{false, false, 0.0, 0.0, 0, 0u};
  const int64_t e = p.perm ? p.perm[j] : j;
  const int32_t r = p.row[e], a = p.i0[e], b = p.i1[e];
  const int32_t tag = (dest_of(p, e) % p.group_rows) << kTagShift;
  // no values (matrix-free ph-ph weights, recomputed at every right-hand
  // side): stored weights are 0, so they set no mixed-precision block scale
  const double v = p.val ? p.val[e] : 0.0;
  if (p.kind == 2) {  // ph-ph: row l, partners a, b
    const double w = p.hw[r], wa = p.hw[a], wb = p.hw[b];
    if (w < p.hw_cut || wa < p.hw_cut || wb < p.hw_cut) return k;
    const double x_em = -w + wa + wb;
    const double x_ab = w - wa + wb;
    k.em = fabs(x_em) <= p.cut;
    k.ab = fabs(x_ab) <= p.cut;
    // emission is symmetric in the two partners: with a mirror-symmetric list
    // one channel of twice the weight stands for (l; a, b) and (l; b, a)
    if (p.fold_em && a > b) k.em = false;
    if (k.em) k.wem = (p.fold_em && a < b ? 2.0 : 1.0) * p.pre * v * gdelta(x_em, p.sigma);
    if (k.ab) k.wab = p.pre2 * v * gdelta(x_ab, p.sigma);
    const int64_t base = p.y_off + p.n_el;
    k.o0 = (int32_t)(base + a) | tag;
    k.o1 = (uint32_t)(base + b);
    return k;
  }
  // e-ph entry: electron r -> electron a (partner) with phonon b
  const double w = p.hw[b];
  if (w < p.hw_cut) return k;
  const double x_em = p.eps[r] - w - p.eps[a];
  const double x_ab = p.eps[r] + w - p.eps[a];
  if (p.kind == 0) {
    k.em = fabs(x_em) <= p.cut;
    k.ab = fabs(x_ab) <= p.cut;
    if (k.em) k.wem = p.pre * v * gdelta(x_em, p.sigma);
    if (k.ab) k.wab = p.pre * v * gdelta(x_ab, p.sigma);
    k.o0 = (int32_t)(p.y_off + a) | tag;
    k.o1 = (uint32_t)(p.y_off + p.n_el + b);
  } else {  // ph-e: the absorption process seen from the phonon
    k.ab = fabs(x_ab) <= p.cut;
    if (k.ab) k.wab = p.pre * v * gdelta(x_ab, p.sigma);
    k.o0 = (int32_t)(p.y_off + r) | tag;
    k.o1 = (uint32_t)(p.y_off + a);
  }
  return k;
}

__global__ __launch_bounds__(256) void k_prep(PrepArgs p, int fill) {
  const int lane = threadIdx.x & 63;
  const int64_t grp = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (grp >= p.n_dest) return;
  const int64_t lo = p.raw_ptr[grp], hi = p.raw_ptr[grp + 1];
  int64_t pos = fill ? p.base[grp] : 0;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int64_t j0 = lo; j0 < hi; j0 += 64) {
    const int64_t j = j0 + lane;
    Kept k{false, false, 0.0, 0.0, 0, 0u};
    if (j < hi) k = classify(p, j);
    const unsigned long long bem = __ballot(k.em), bab = __ballot(k.ab);
    if (fill) {
      int64_t my = pos + __popcll(bem & below) + __popcll(bab & below);
      if (k.em) { p.out[my] = Channel{k.o0, k.o1 | kEmBit, k.wem}; ++my; }
      if (k.ab) p.out[my] = Channel{k.o0, k.o1, k.wab};
    }
    pos += __popcll(bem) + __popcll(bab);
  }
  if (!fill && lane == 0) p.count[grp] = pos;
}

hipError_t launch_prep_count(const PrepArgs& p, hipStream_t s) {
  if (p.n_dest == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prep, dim3((unsigned)((p.n_dest + 3) / 4)), dim3(256), 0, s, p, 0);
  return hipGetLastError();
}

hipError_t launch_prep_fill(const PrepArgs& p, hipStream_t s) {
  if (p.n_dest == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prep, dim3((unsigned)((p.n_dest + 3) / 4)), dim3(256), 0, s, p, 1);
  return hipGetLastError();
}

// ---------------------------------------------------------------- observables
// Energy-resolved averages: one wavefront per bin reduces the populations of
// the bin's states (idx[ptr[b] .. ptr[b+1])) in a fixed order.  out[3b] = state
// count, out[3b+1] = mean population, out[3b+2] = mean of (y - y_ref) (0 when
// y_ref is null).
__global__ __launch_bounds__(64) void k_bin_means(const double* __restrict__ y, const double* __restrict__ yref,
                                                  const int32_t* idx, const int32_t* ptr, int n_bins, double* out) {
  const int b = blockIdx.x;
  if (b >= n_bins) return;
  const int lane = threadIdx.x;
  double sp = 0.0, sd = 0.0;
  for (int32_t k = ptr[b] + lane; k < ptr[b + 1]; k += 64) {
    const double v = y[idx[k]];
    sp += v;
    if (yref) sd += v - yref[idx[k]];
  }
  for (int o = 32; o > 0; o >>= 1) {
    sp += __shfl_xor(sp, o, 64);
    sd += __shfl_xor(sd, o, 64);
  }
  if (lane == 0) {
    const int32_t n = ptr[b + 1] - ptr[b];
    out[3 * b] = (double)n;
    out[3 * b + 1] = n ? sp / n : 0.0;
    out[3 * b + 2] = n ? sd / n : 0.0;
  }
}

hipError_t launch_bin_means(const double* y, const double* yref, const int32_t* idx, const int32_t* ptr,
                            int n_bins, double* out, hipStream_t s) {
  if (n_bins <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bin_means, dim3((unsigned)n_bins), dim3(64), 0, s, y, yref, idx, ptr, n_bins, out);
  return hipGetLastError();
}

// Effective temperature of each phonon branch: the T at which Bose-Einstein
// occupations of the branch's states carry the branch's energy sum hw N.
// One block per branch; bisection in log T over [1e-2, 1e7] K, every sum a
// fixed-order block reduction.  States with hw <= 0 are left out.
__device__ __forceinline__ double block_sum256(double v, double* red) {
  const int t = threadIdx.x;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_mode_temperature(const double* __restrict__ y, const double* __restrict__ e,
                                                          const int32_t* idx, const int32_t* ptr, int n_modes,
                                                          double* T_out) {
  __shared__ double red[4];
  const int m = blockIdx.x;
  if (m >= n_modes) return;
  const double kB = 8.617333262e-5;   // eV/K
  double v = 0.0;
  for (int32_t k = ptr[m] + threadIdx.x; k < ptr[m + 1]; k += 256) {
    const double w = e[idx[k]];
    if (w > 0.0) v += w * y[idx[k]];
  }
  const double target = block_sum256(v, red);
  if (!(target > 0.0)) {
    if (threadIdx.x == 0) T_out[m] = 0.0;
    return;
  }
  double lo = log(1e-2), hi = log(1e7);
  for (int it = 0; it < 100; ++it) {
    const double mid = 0.5 * (lo + hi);
    const double kT = kB * exp(mid);
    double u = 0.0;
    for (int32_t k = ptr[m] + threadIdx.x; k < ptr[m + 1]; k += 256) {
      const double w = e[idx[k]];
      if (w > 0.0) u += w / expm1(w / kT);
    }
    const double tot = block_sum256(u, red);
    if (tot < target) lo = mid;
    else hi = mid;
  }
  if (threadIdx.x == 0) T_out[m] = exp(0.5 * (lo + hi));
}

hipError_t launch_mode_temperature(const double* y, const double* e, const int32_t* idx, const int32_t* ptr,
                                   int n_modes, double* T_out, hipStream_t s) {
  if (n_modes <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mode_temperature, dim3((unsigned)n_modes), dim3(256), 0, s, y, e, idx, ptr, n_modes, T_out);
  return hipGetLastError();
}

}  // namespace rtbte
