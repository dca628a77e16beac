// Internal declarations shared by the rtbte host code and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rtbte.h"

namespace rtbte {

constexpr double kHbarEvFs = 0.6582119569;          // eV fs
constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrtPi = 1.7724538509055160273;
constexpr uint32_t kEmBit = 0x80000000u;            // channel kind bit: emission
constexpr uint32_t kIdxMask = 0x7fffffffu;
constexpr int32_t kTagShift = 27;                   // row tag inside a group: bits 27..30 of i0
constexpr int32_t kPosMask = 0x07ffffff;            // state index: bits 0..26 of i0 / i1
constexpr int kMaxGroupRows = 16;
constexpr double kHealthTol = 1e-6;                 // occupations checked against [-tol, 1 + tol] / [-tol, inf)

// A stored channel, 16 bytes, streamed once per right-hand-side evaluation.
// Channels of a group of up to 16 consecutive destination rows are stored
// together, merged in partner order; bits 27..30 of i0 say which row of the
// group the channel belongs to.
//   electron rows (I^{e-ph}):  i0 = partner electron s | tag, i1 = phonon p | em bit
//   phonon rows, ph-e range    i0 = electron r | tag,         i1 = electron s (absorption)
//   phonon rows, ph-ph range   i0 = phonon a | tag,           i1 = phonon b | em bit
// Indices are positions in the concatenated state vector y; w already holds
// prefactor * |M|^2 * delta (and the factor 2 of ph-ph absorption).
struct Channel {
  int32_t i0;
  uint32_t i1;
  double w;
};
static_assert(sizeof(Channel) == 16, "channel must be 16 bytes");

// A group of consecutive destination rows of one kind (electron or phonon)
// of one instance, and its channel ranges.
struct Group {
  int64_t start;   // first channel
  int64_t split;   // phonon groups: end of the ph-e channels, start of ph-ph; electron: = end
  int64_t end;
  int32_t row0;    // first row (position in y)
  int32_t inst;
  int32_t nrows;   // 1..16
  int32_t phonon;  // 1: phonon rows
};

// Per-instance integrator state, resident on the device.
struct InstState {
  double t, t_out, t_start, h, h_use, h_cap, e1, e2, eps, h_min, h_max, h0_d0, h0_d1;
  int32_t first, fails, done, status, accepted, last, one_step, need_h0;
  int64_t n_accept, n_reject, n_attempt, n_evals, steps_left;
};

struct InstInfo {
  int64_t off;   // offset of the instance in y
  int32_t n_el, n_ph;
};

// Controller constants (PID of Eq. (pid_controller) and its safeguards).
struct Ctl {
  double k1, k2, k3, order, safety, eta_max, eta_max_first, eta_fail_min, eta_fail_max, eps_floor;
  double eta_fail_repeat;              // ratio cap from the small_nef-th consecutive failure on
  double rtol, atol_el, atol_ph;
  int32_t max_fails, alt_sign, fixed;  // fixed: fixed step, every step accepted
  int32_t small_nef;
  int32_t stages;                      // right-hand-side evaluations per attempt
};

// A work item: a bounded range of one group's channels, streamed by one
// wavefront, which writes the item's sum for every row of the group.
struct Item {
  int64_t lo, hi;  // channel range, inside [start, end) of its group
  int32_t group;
  int32_t pad;
};

// Tiled launch (packed channel formats).  A segment is the channels of one
// kind in one group (electron groups: e-ph; phonon groups: ph-e, then ph-ph),
// stored merged by one partner, the key (e-ph: the phonon; ph-e: the
// initial electron; ph-ph: the first phonon).  Its items are cut where the
// key crosses a multiple of the key block length, and a launch block holds
// up to kTileWaves such items, from consecutive groups of one kind of one
// instance with the same key block.  The block stages in LDS the
// populations of its key block and of a window of the other partner's
// positions (the span its channels touch, up to the window capacity), so
// most gathers of a channel read LDS; an other partner outside the window
// is gathered from global memory.
// A block runs through a range of key blocks; its waves keep their row sums
// across the range and write one item each at the end.
constexpr int kTileWaves = 4;
constexpr int kTileKey64 = 1024, kTileOther64 = 2944;    // FP64 staging capacities (states)
constexpr int kTileKey32 = 2048, kTileOther32 = 4096;    // mixed (4-byte population codes)
constexpr uint32_t kTileEmpty = 0xffffffffu;             // Tile.lo of a key block with no channels
struct TileBlock {
  int64_t bndo[kTileWaves];  // offset of each wave's segment in the key-block bounds (-1: none)
  int32_t item[kTileWaves];  // item (row-sum slot) of each wave (-1: none)
  int32_t inst;
  int32_t kind;              // 0 e-ph, 1 ph-e, 2 ph-ph
  int32_t j0, j1;            // key blocks [j0, j1)
  int32_t tile0;             // tile of key block j0 (the tiles of j0..j1-1 follow it)
  int32_t pad;
};
static_assert(sizeof(TileBlock) == 72, "tile block record");
// The staged window of the other partner in one key block of one set of
// groups: positions [lo, lo + len) relative to the instance (lo = kTileEmpty:
// no channels in this key block).
struct Tile {
  uint32_t lo, len;
};

// Matrix-free ph-ph weights of one instance: the rtbte_pp_model, the
// instance's ph-ph prefactor over the delta's normalisation sigma sqrt(pi),
// the reciprocal width, whether its emission pairs are folded, where its
// phonons start, and FP64 reciprocals of the branch count and grid side
// (the kernel divides phonon ids by them).
struct PpModel {
  int32_t dim, L, n_modes, folded;
  uint32_t key0, key1, stream, n_el;
  double ln_mu, ln_sigma, pre_norm, rcp_sigma, rcp_modes, rcp_L;
};

// Arguments of the collision kernel (per-item row sums).
// FP64 channels, packed (12 bytes): an 8-byte word per channel, low half
// pos0 (bits 0..P-1) | tag (P..P+3) | weight field bits 32..59-P (P+4..31),
// high half pos1 (0..P-1) | em (P) | weight field bits 60-P.. (P+1..31), and
// a 4-byte word with weight field bits 0..31; positions relative to the
// instance; the weight field is the FP64 bit pattern without its sign and its
// 52 - M lowest mantissa bits, M = min(80 - 2P, 52) (rounded to nearest).
struct RowArgs {
  const Channel* ch;        // 16-byte channels (nullptr when packed)
  const uint64_t* pk;       // packed: [n_ch] 8-byte words
  const uint32_t* pkw;      // packed: [n_ch] low weight words
  int32_t pack_p, pack_m;   // packed: position bits P, mantissa bits M
  const InstInfo* info;     // packed: instance offsets
  const Group* groups;
  const Item* items;
  const int32_t* order;     // [n_items] processing order (longest first)
  int64_t n_items;
  int32_t parts;
  const double* z;          // populations the integrals are evaluated at
  double* partial;          // [n_items][kMaxGroupRows] row sums of each item
  const InstState* st;      // stage mode: items of finished instances are skipped (else nullptr)
  int32_t deriv;            // 1: each term is -W dF/dx_row (the rows then hold linearized rates)
  const TileBlock* blocks;  // tiled launch (packed layout): [n_blocks], else nullptr
  const int32_t* border;    // [n_blocks] processing order of the blocks
  int64_t n_blocks;
  const Tile* tiles;
  const int64_t* bnd;       // key-block bounds of every segment
  int64_t ny;               // length of z
  const PpModel* ppm;       // matrix-free ph-ph weights: [n_inst] models (else nullptr)
  const double* hw;         // [ny] state energies (phonons: hbar omega), with ppm
};

// Arguments of the row kernel: sums of the items of each row's group, the
// sign of the collision integral, and the plain or ERK-stage epilogue.
struct FinishArgs {
  const Group* groups;
  const int32_t* row_group; // [n_rows] group of each row
  const int64_t* item_ptr;  // [n_groups + 1] items of each group
  const double* partial;
  int64_t n_rows;
  double* out;              // plain mode: f(z)
  // stage mode
  const double* y;          // y_{n-1}
  double* k[5];             // stage derivatives k_j (k[stage] written)
  double* zout;             // next stage state (not last)
  double* ynew;             // last stage: candidate solution
  double* lte;              // last stage: local error estimate
  const double* forcing;    // MIS forcing added on phonon rows, or nullptr
  const InstState* st;
  double a[5], b[5], d[5];  // z_{i+1} = y + h sum_j a_j k_j; ynew = y + h sum b_j k_j; lte = h sum d_j k_j
  int32_t stage, last;
};

// Launchers (kernels.hip)
hipError_t launch_items(const RowArgs& a, int slots, hipStream_t s);
hipError_t launch_pack12(const Channel* ch, int64_t n_ch, const Group* groups, int64_t n_groups,
                         const InstInfo* info, int p_bits, int m_bits, uint64_t* pk, uint32_t* pkw, hipStream_t s);
hipError_t launch_finish_rows(const FinishArgs& f, bool stage, hipStream_t s);

// Mixed precision: weights relative to one FP32 scale per block of kMixBlock
// consecutive channels, populations as 4-byte codes.
// 10-byte formats: index word x = pos0 (bits 0..23) | tag (24..27) | tail
// bits 0..3 (28..31); y = pos1 (0..23) | tail bits 4..10 (24..30) | em (31),
// plus a 16-bit weight head; the 11-bit tail extends an FP16 weight's
// significand (RTBTE_W_F16X), it is zero in the other 10-byte formats.
// 8-byte format (RTBTE_W_PACK8), P-bit positions relative to the instance:
// x = pos0 (0..P-1) | tag (P..P+3) | weight bits 0..27-P (P+4..31);
// y = pos1 (0..P-1) | weight bits 28-P.. (P..30) | em (31); the weight is a
// small float of 6 exponent bits over M = min(53 - 2P, 23) mantissa bits
// (the field's spare high bits are zero).
constexpr int kMixBlock = 512;
constexpr int32_t kMixPosMask = 0x00ffffff;
constexpr int32_t kMixTagShift = 24;
struct MixArgs {
  const int2* idx;          // [n_ch] packed as above
  const uint16_t* wq;       // [n_ch] weight / scale of its block, 16-bit head
  const float* scale;       // [n_scale] = [ceil(n_ch / kMixBlock)]
  int64_t n_scale;
  const float* pop;         // [ny] one coded FP32 word per state (k_popf)
  const Group* groups;
  const Item* items;
  const int32_t* order;
  int64_t n_items;
  int32_t parts;
  int32_t wfmt;             // RTBTE_W_* weight format (never RTBTE_W_AUTO here)
  int32_t pack_p, pack_m;   // RTBTE_W_PACK8: position bits P, mantissa bits M
  const InstInfo* info;     // RTBTE_W_PACK8: instance offsets
  double* partial;
  const InstState* st;
  const TileBlock* blocks;  // tiled launch (RTBTE_W_PACK8), else nullptr
  const int32_t* border;
  int64_t n_blocks;
  const Tile* tiles;
  const int64_t* bnd;
  int64_t ny;
  const PpModel* ppm;
  const double* hw;
};
hipError_t launch_items_mixed(const MixArgs& a, int slots, hipStream_t s);
// Tiled launches (create time), from the packed 8-byte words (FP64 or
// mixed; positions in the low P bits of each half): for each segment, the
// first channel whose key reaches j * key_len, j = 0..n_kb, at
// bnd[off + j]; and for each (set of up to kTileWaves segments, key block),
// the smallest and largest other-partner position of its channels.
struct SegRange {
  int64_t lo, hi;     // channels [lo, hi)
  int64_t off;        // its bounds start at bnd[off]
  int32_t kind;       // 0 e-ph (key: second partner), 1 ph-e, 2 ph-ph (key: first partner)
  int32_t n_kb;       // key blocks
};
hipError_t launch_key_bounds(const uint64_t* words, int pack_p, const SegRange* segs, int64_t n_segs,
                             int64_t key_len, int64_t* bnd, hipStream_t s);
struct SpanJob {
  int64_t bndo[kTileWaves];   // bounds of each segment of the set (-1: none)
  int32_t j;                  // key block
  int32_t kind;
};
hipError_t launch_tile_span(const uint64_t* words, int pack_p, const SpanJob* jobs, int64_t n_jobs,
                            const int64_t* bnd, uint32_t* span, hipStream_t s);
// pop[i] from z[i] (each factor formed in FP64, then rounded to FP32)
hipError_t launch_popf(float* pop, const double* z, const int32_t* row_group, const Group* groups,
                       int64_t n, hipStream_t s);
// create time: per-block scales, then the 16-bit weights and packed indices
hipError_t launch_mix_scales(const Channel* ch, int64_t n_ch, float headroom, float* scale, hipStream_t s);
hipError_t launch_mix_convert(const Channel* ch, int64_t n_ch, const Group* groups, int64_t n_groups,
                              const float* scale, int wfmt, int2* idx, uint16_t* wq, hipStream_t s);
hipError_t launch_mix_pack8(const Channel* ch, int64_t n_ch, const Group* groups, int64_t n_groups,
                            const InstInfo* info, const float* scale, int p_bits, int m_bits, int2* words,
                            hipStream_t s);
hipError_t launch_wrms(const double* v, const double* y, const InstInfo* info, const InstState* st,
                       double* partial, int n_inst, int nchunk, Ctl c, hipStream_t s);
hipError_t launch_control(InstState* st, const double* partial, const InstInfo* info, int n_inst,
                          int nchunk, Ctl c, hipStream_t s);
hipError_t launch_commit(double* y, const double* ynew, const int32_t* row_inst,
                         const InstState* st, int64_t n, hipStream_t s);
// health[inst] |= 1 when an electron occupation of y leaves [-tol, 1 + tol]
// (or is not a number), |= 2 when a phonon occupation is below -tol (or not a
// number); one block per instance
hipError_t launch_health(const double* y, const InstInfo* info, int32_t* health, int n_inst, double tol,
                         hipStream_t s);
hipError_t launch_begin(InstState* st, const double* t_in, const double* h_in, int n_inst,
                        double t_out, int one_step, double h_cap, int64_t fixed_steps,
                        double fixed_h, hipStream_t s);
hipError_t launch_finish(const InstState* st, double* t_out_buf, double* h_out_buf, int n_inst,
                         int32_t* summary, hipStream_t s);
hipError_t launch_h0_stage1(InstState* st, const double* partial_y, const double* partial_f,
                            const InstInfo* info, int n_inst, int nchunk, hipStream_t s);
hipError_t launch_h0_axpy(double* out, const double* y, const double* f, const int32_t* row_inst,
                          const InstState* st, int64_t n, hipStream_t s);
hipError_t launch_sub(double* out, const double* a, const double* b, int64_t n, hipStream_t s);
hipError_t launch_h0_stage2(InstState* st, const double* partial_d, const InstInfo* info, int n_inst,
                            int nchunk, double order, hipStream_t s);
hipError_t launch_lincomb(double* out, const double* const* vecs, const double* coef, int nv,
                          int64_t off, int64_t n, hipStream_t s);

// Create-time channel preparation (kernels.hip)
struct PrepArgs {
  // raw entries of one instance (device), visited through perm (nullptr: identity)
  const int32_t* row;
  const int32_t* i0;
  const int32_t* i1;
  const double* val;
  const int64_t* perm;
  const int64_t* raw_ptr;   // [n_dest + 1] raw entries of each destination group (in visiting order)
  int32_t n_dest;           // destination groups
  int32_t group_rows;       // rows per group (groups start at multiples of it)
  const double* eps;        // instance band energies (device)
  const double* hw;         // instance phonon energies (device)
  double sigma, cut, pre, pre2, hw_cut;
  int64_t y_off;            // instance offset in y
  int32_t n_el;
  int32_t kind;             // 0 e-ph electron side, 1 ph-e, 2 ph-ph
  int32_t fold_em;          // ph-ph: store the emission channel of (l; a, b), a < b, with twice
                            // its weight for itself and its mirror (l; b, a), which gives none
  int64_t* count;           // [n_dest] kept channels per group (count pass)
  const int64_t* base;      // [n_dest] first output slot of each group (fill pass)
  Channel* out;
};
hipError_t launch_prep_count(const PrepArgs& p, hipStream_t s);
hipError_t launch_prep_fill(const PrepArgs& p, hipStream_t s);

// observables
hipError_t launch_bin_means(const double* y, const double* yref, const int32_t* idx, const int32_t* ptr,
                            int n_bins, double* out, hipStream_t s);
hipError_t launch_mode_temperature(const double* y, const double* e, const int32_t* idx, const int32_t* ptr,
                                   int n_modes, double* T_out, hipStream_t s);

}  // namespace rtbte
