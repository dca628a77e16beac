// rtbte C ABI: context creation (channel preparation), right-hand side, and
// the device-driven integrators (adaptive ERK, fixed RK4, MIS multirate).
//
// Host code here does bookkeeping only: argument checks, integer grouping of
// the input entries by destination row, buffer management, and the launch
// sequence.  Every floating-point step of the method -- channel weights,
// collision integrals, stage updates, error norms, step control -- runs in the
// kernels of kernels.hip.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include <rocprofiler-sdk-roctx/roctx.h>
#include <string>
#include <vector>

#include "rtbte.h"
#include "internal.h"

using namespace rtbte;

namespace rtbte {
hipError_t launch_diff_norms(const double* a, const double* b, const InstInfo* info, double* partial, int n_inst,
                             int nchunk, hipStream_t s);
hipError_t launch_fill(double* p, double v, int64_t n, hipStream_t s);
hipError_t launch_select_max_norm(const double* partial, const InstInfo* info, int n_inst, int nchunk,
                                  double* sel_partial, InstInfo* sel_info, hipStream_t s);
hipError_t launch_broadcast_first(double* p, int64_t n, hipStream_t s);
}

// A roctx range over a library call or a poll interval, shown by
// `rocprofv3 --marker-trace` beside the kernels it enqueued (a host-side
// marker: no stream work, nothing recorded into captured graphs).
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePush(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

namespace {

thread_local std::string g_create_error;

// Zonneveld 5-stage pair (main order 4, embedding order 3), the default ERK of
// the integrators the paper uses (Methods, ERK method).
const double ZA[5][5] = {{0, 0, 0, 0, 0},
                         {0.5, 0, 0, 0, 0},
                         {0, 0.5, 0, 0, 0},
                         {0, 0, 1.0, 0, 0},
                         {5.0 / 32, 7.0 / 32, 13.0 / 32, -1.0 / 32, 0}};
const double ZB[5] = {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6, 0.0};
const double ZBT[5] = {-0.5, 7.0 / 3, 7.0 / 3, 13.0 / 6, -16.0 / 3};

// Classical RK4.
const double RA[4][4] = {{0, 0, 0, 0}, {0.5, 0, 0, 0}, {0, 0.5, 0, 0}, {0, 0, 1.0, 0}};
const double RB[4] = {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6};

// MIS with the Knoth-Wolke 3-stage base method: abscissae c_hat = (0, 1/3, 3/4, 1)
// and the constant forcing of stage i, r_i = sum_j (Omega_ij / dc_i) f^s(z_j),
// Omega from Eq. (mis_coef) (last row b_j - A_{S,j}).
const double MIS_C[4] = {0.0, 1.0 / 3, 3.0 / 4, 1.0};
const double MIS_R[4][3] = {{0, 0, 0},
                            {1.0, 0, 0},
                            {-5.0 / 4, 9.0 / 4, 0},
                            {17.0 / 12, -51.0 / 20, 32.0 / 15}};

struct Tableau {
  int S;
  double A[5][5], b[5], d[5];
  bool embedded;
};

Tableau zonneveld() {
  Tableau t{};
  t.S = 5;
  for (int i = 0; i < 5; ++i) {
    for (int j = 0; j < 5; ++j) t.A[i][j] = ZA[i][j];
    t.b[i] = ZB[i];
    t.d[i] = ZB[i] - ZBT[i];
  }
  t.embedded = true;
  return t;
}

Tableau rk4() {
  Tableau t{};
  t.S = 4;
  for (int i = 0; i < 4; ++i) {
    for (int j = 0; j < 4; ++j) t.A[i][j] = RA[i][j];
    t.b[i] = RB[i];
    t.d[i] = 0.0;
  }
  t.embedded = false;
  return t;
}

template <class T>
T* dalloc(size_t n, hipError_t* err) {
  void* p = nullptr;
  *err = hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T));
  return static_cast<T*>(p);
}

// Scratch of the allocation-free right-hand side (rtbte_rhs_noalloc): the
// per-item row sums of one evaluation and, in mixed precision, the
// population codes after them.  Every device the library runs on holds its
// own copy until the process ends.  In host code `scratch` names a host-side
// stand-in, never the device memory: its device address is taken once per
// device with hipGetSymbolAddress (scratch_setup) and only that address is
// passed to kernels.
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_dev;   // device address of `scratch`, per device (null: not taken yet)

// With `device` current: its address of `scratch` (taken on first use).
hipError_t scratch_setup(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= device) g_scratch_dev.resize((size_t)device + 1, nullptr);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[device] = p;
  }
  *out = g_scratch_dev[device];
  return hipSuccess;
}

// Bytes of static scratch one right-hand side of this shape needs: the item
// row sums (rounded up to 256 B), then the FP32 population codes (mixed).
size_t noalloc_scratch_bytes(int64_t n_items, int64_t ny, bool mixed) {
  const size_t sums = (((size_t)std::max<int64_t>(n_items, 1) * kMaxGroupRows * sizeof(double)) + 255) & ~(size_t)255;
  return sums + (mixed ? (size_t)ny * sizeof(float) : 0);
}

}  // namespace

struct rtbte_ctx {
  int device = 0;
  rtbte_options opt{};
  std::string err;
  int n_inst = 0;
  std::vector<InstInfo> info;
  int64_t ny = 0;
  std::vector<int64_t> counts;     // [3 * n_inst]
  int64_t n_ch = 0;
  int64_t n_groups = 0;
  int64_t n_items = 0;
  int group_rows_el = 8, group_rows_ph = 16;
  int64_t item_channels = 0;
  int slots = 16;
  int nchunk = 1;
  // device
  Channel* ch = nullptr;
  Group* groups = nullptr;
  Item* items = nullptr;
  int32_t* order = nullptr;       // item processing order
  int64_t* item_ptr = nullptr;    // [n_groups + 1]
  int32_t* row_group = nullptr;   // [ny]
  double* partial_items = nullptr;
  // mixed precision
  bool mixed = false;
  int wfmt = -1;                  // weight format in use (RTBTE_W_*); FP64: -1 plain, -2 packed
  int pack_p = 0, pack_m = 0;     // packed layouts: position and mantissa bits
  int f64_m = 0;                  // FP64 packed lists: mantissa bits kept
  bool keep64 = false;            // a mixed context that also holds the FP64 lists
  std::vector<double> err64;      // [n_inst] last mixed-vs-FP64 right-hand-side difference (-1: none)
  std::vector<int64_t> folded;    // [n_inst] ph-ph emission channels stored in their mirror's weight
  int64_t polls = 0;              // polls since the last periodic FP64 check
  uint64_t* pk = nullptr;         // FP64 packed: 8-byte words
  uint32_t* pkw = nullptr;        // FP64 packed: low weight words
  int2* mix_idx = nullptr;
  uint16_t* mix_wq = nullptr;
  float* mix_scale = nullptr;
  float* popf = nullptr;
  int32_t* row_inst = nullptr;
  InstInfo* info_d = nullptr;
  InstState* st = nullptr;       // main integrator
  InstState* st_fast = nullptr;  // MIS fast integrator
  InstState* st_slow = nullptr;  // MIS slow-step controller (adaptive multirate; one entry)
  double* mra = nullptr;         // [3 * ny + nchunk + 2] adaptive multirate: full-step, half-step and
                                 // estimate vectors, then the selected instance's WRMS partials and sizes
  double* mis_keep = nullptr;    // [ny] multirate: the state at the start of the current slow step
  double* kbuf[5] = {};
  double* zb[2] = {};
  double* ynew = nullptr;
  double* lte = nullptr;
  double* tmp = nullptr;
  double* tmp2 = nullptr;
  double* fs[3] = {};
  double* forcing = nullptr;
  double* partial = nullptr;     // [3][n_inst * nchunk]
  double* tvec = nullptr;        // [2 * n_inst] scratch t / h for inner solves
  int32_t* summary_d = nullptr;
  int32_t* summary_h = nullptr;  // pinned
  double* scal_h = nullptr;      // pinned host scalars
  // host tallies of right-hand-side evaluations outside the predicated step loop
  int64_t extra_rhs[3] = {0, 0, 0};
  int64_t slow_steps = 0;
  int64_t split_slow_evals = 0;  // ph-ph evaluations of operator-splitting steps (run on st_fast)
  int last_status = 0;
  // timing of the collision-kernel launches with HIP events on their stream
  bool prof = false;
  struct Pending { hipEvent_t a, b; double bytes; };
  std::vector<Pending> pending;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  double prof_ms = 0.0, prof_bytes = 0.0;
  int64_t prof_n = 0;
  // host copy of the group table (work items are cut from it)
  std::vector<Group> groups_h;
  // state energies (eV): eps of the electron states, hbar omega of the phonons
  std::vector<double> energy_h;
  double* energy_d = nullptr;
  // captured step sequences, replayed through HIP graphs (use_graph)
  struct GraphKey {
    const double* y; const double* forcing; const InstState* st;
    int tb_stages, parts, steps;   // the tableau is identified by its stage count (RK4 4, Zonneveld 5)
    Ctl ctl;
  };
  struct GraphEntry { GraphKey key; hipGraph_t g; hipGraphExec_t exec; };
  std::vector<GraphEntry> graphs;
  hipStream_t cap = nullptr;       // capture stream (default priority)
  int64_t graph_launches = 0;
  // launch-shape tuning: source of the shape and the time it measured
  int tuned = 0;                   // 0 given/default, 1 measured at create, 2 from the cache
  double tuned_ms = 0.0;
  // this device's address of the static scratch (rtbte_rhs_noalloc)
  void* scratch_dev = nullptr;
  // matrix-free ph-ph weights: one model per instance (device)
  PpModel* ppm = nullptr;
  // tiled launch (packed layouts): blocks, their order, tiles, key-block bounds
  bool tiled = false;
  TileBlock* tblocks = nullptr;
  int32_t* border = nullptr;
  Tile* tiles = nullptr;
  int64_t* bnd = nullptr;
  int64_t n_blocks = 0;
  double tile_in_window = 0.0;    // fraction of tiles whose other partners are staged
  int32_t* health = nullptr;      // [n_inst] RTBTE_HEALTH_* bits since create / reset
};

static int fail(rtbte_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  else g_create_error = buf;
  return code;
}

#define HIPCHK(ctx, expr)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail((ctx), e_ == hipErrorOutOfMemory ? RTBTE_E_NOMEM : RTBTE_E_HIP, "%s: %s", \
                  #expr, hipGetErrorString(e_));                                           \
  } while (0)

extern "C" {

void rtbte_default_options(rtbte_options* o) {
  std::memset(o, 0, sizeof *o);
  o->precision = RTBTE_FP64;
  o->device = 0;
  o->rtol = 1e-6;
  o->atol_el = 1e-9;
  o->atol_ph = 1e-12;
  o->fast_mode = 0;
  o->h_fast = 1.0;
  o->fast_rtol = 1e-5;
  o->fast_atol_el = 1e-9;
  o->fast_atol_ph = 1e-11;
  o->pid_k1 = 0.58;
  o->pid_k2 = 0.21;
  o->pid_k3 = 0.10;
  o->pid_order = 4;
  o->pid_alt_sign = 0;
  o->safety = 0.96;
  o->eta_max = 20.0;
  o->eta_max_first = 1e4;
  o->eta_fail_min = 0.1;
  o->eta_fail_max = 0.9;
  o->eps_floor = 1e-10;
  o->max_fails = 7;
  o->use_graph = 0;
  o->steps_per_poll = 8;
  o->group_rows_el = 0;
  o->group_rows_ph = 0;
  o->item_channels = 0;
  o->mixed_weights = RTBTE_W_AUTO;
  o->tune = 0;
  o->tune_cache = nullptr;
  o->fp64_layout = RTBTE_F64_AUTO;
  o->fp64_check = 0;
  o->small_nef = 5;
  o->eta_fail_repeat = 0.3;
  o->pp_fold = 1;
  o->tiled = 0;
}

const char* rtbte_last_error(const rtbte_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

}  // extern "C"

// ---------------------------------------------------------------- create
namespace {

// Visiting order of n raw entries for the channel preparation: grouped by
// destination group dest[i] / G (stable counting sort), and inside a group
// with more than one row merged by `key` (stable: ties keep input order).
// Returns the permutation (empty if it is the identity) and the group pointers.
void group_entries(int64_t n, const int32_t* dest, int32_t nrows, int G, const int32_t* key,
                   std::vector<int64_t>& perm, std::vector<int64_t>& gptr) {
  const int32_t ng = (nrows + G - 1) / G;
  gptr.assign((size_t)ng + 1, 0);
  bool sorted = true;
  for (int64_t i = 0; i < n; ++i) {
    gptr[(size_t)(dest[i] / G) + 1]++;
    if (i && dest[i] / G < dest[i - 1] / G) sorted = false;
  }
  for (int32_t k = 0; k < ng; ++k) gptr[k + 1] += gptr[k];
  perm.clear();
  if (sorted && G == 1) return;
  perm.resize((size_t)n);
  const int nt = std::max(1, omp_get_max_threads());
  if (sorted) {
#pragma omp parallel for num_threads(nt)
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
  } else {
    // per-thread histograms over contiguous chunks keep the order stable
    std::vector<std::vector<int64_t>> cur((size_t)nt);
    const int64_t chunk = (n + nt - 1) / nt;
#pragma omp parallel num_threads(nt)
    {
      const int t = omp_get_thread_num();
      std::vector<int64_t>& h = cur[t];
      h.assign((size_t)ng, 0);
      const int64_t lo = std::min(n, t * chunk), hi = std::min(n, lo + chunk);
      for (int64_t i = lo; i < hi; ++i) h[dest[i] / G]++;
    }
    for (int32_t k = 0; k < ng; ++k) {
      int64_t pos = gptr[k];
      for (int t = 0; t < nt; ++t) {
        int64_t c = cur[t][k];
        cur[t][k] = pos;
        pos += c;
      }
    }
#pragma omp parallel num_threads(nt)
    {
      const int t = omp_get_thread_num();
      std::vector<int64_t>& h = cur[t];
      const int64_t lo = std::min(n, t * chunk), hi = std::min(n, lo + chunk);
      for (int64_t i = lo; i < hi; ++i) perm[h[dest[i] / G]++] = i;
    }
  }
  if (G > 1) {
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
    for (int32_t g = 0; g < ng; ++g)
      std::stable_sort(perm.begin() + gptr[g], perm.begin() + gptr[g + 1],
                       [&](int64_t x, int64_t y) { return key[x] < key[y]; });
  }
}

int check_problem(const rtbte_problem& p, int inst, bool v2_optional = false) {
  if (p.n_el < 0 || p.n_ph < 0 || p.n_eph < 0 || p.n_pp < 0)
    return fail(nullptr, RTBTE_E_INVAL, "instance %d: negative size", inst);
  if ((int64_t)p.n_el + p.n_ph == 0)
    return fail(nullptr, RTBTE_E_INVAL, "instance %d: no states (n_el + n_ph must be > 0)", inst);
  if (p.n_k_total <= 0 || p.n_q_total <= 0)
    return fail(nullptr, RTBTE_E_INVAL, "instance %d: n_k_total and n_q_total must be > 0", inst);
  if (!(p.sigma_eph > 0) || !(p.sigma_pp > 0) || !(p.nsigma > 0))
    return fail(nullptr, RTBTE_E_INVAL, "instance %d: sigma and nsigma must be > 0", inst);
  if ((p.n_el && !p.eps) || (p.n_ph && !p.hw))
    return fail(nullptr, RTBTE_E_INVAL, "instance %d: missing energies", inst);
  if (p.n_eph && (!p.eph_row || !p.eph_partner || !p.eph_phonon || !p.eph_g2))
    return fail(nullptr, RTBTE_E_INVAL, "instance %d: missing e-ph arrays", inst);
  if (p.n_pp && (!p.pp_row || !p.pp_a || !p.pp_b || (!p.pp_v2 && !v2_optional)))
    return fail(nullptr, RTBTE_E_INVAL, "instance %d: missing ph-ph arrays", inst);
  int64_t bad = -1;
#pragma omp parallel for reduction(max : bad)
  for (int64_t i = 0; i < p.n_eph; ++i)
    if (p.eph_row[i] < 0 || p.eph_row[i] >= p.n_el || p.eph_partner[i] < 0 ||
        p.eph_partner[i] >= p.n_el || p.eph_phonon[i] < 0 || p.eph_phonon[i] >= p.n_ph)
      bad = std::max(bad, i);
  if (bad >= 0) return fail(nullptr, RTBTE_E_INVAL, "instance %d: e-ph entry %lld out of range", inst, (long long)bad);
#pragma omp parallel for reduction(max : bad)
  for (int64_t i = 0; i < p.n_pp; ++i)
    if (p.pp_row[i] < 0 || p.pp_row[i] >= p.n_ph || p.pp_a[i] < 0 || p.pp_a[i] >= p.n_ph ||
        p.pp_b[i] < 0 || p.pp_b[i] >= p.n_ph)
      bad = std::max(bad, i);
  if (bad >= 0) return fail(nullptr, RTBTE_E_INVAL, "instance %d: ph-ph entry %lld out of range", inst, (long long)bad);
  return RTBTE_OK;
}

struct DevRaw {
  int32_t *er = nullptr, *es = nullptr, *ep = nullptr, *pr = nullptr, *pa = nullptr, *pb = nullptr;
  double *eg = nullptr, *pv = nullptr, *eps = nullptr, *hw = nullptr;
  int64_t *perm_e = nullptr, *perm_pe = nullptr, *perm_pp = nullptr;
  int64_t *ptr_e = nullptr, *ptr_pe = nullptr, *ptr_pp = nullptr;
  int64_t *cnt_e = nullptr, *cnt_pe = nullptr, *cnt_pp = nullptr;
  int64_t *base_e = nullptr, *base_pe = nullptr, *base_pp = nullptr;
  void release() {
    void* ps[] = {er, es, ep, pr, pa, pb, eg, pv, eps, hw, perm_e, perm_pe, perm_pp, ptr_e, ptr_pe,
                  ptr_pp, cnt_e, cnt_pe, cnt_pp, base_e, base_pe, base_pp};
    for (void* p : ps)
      if (p) (void)hipFree(p);
    *this = DevRaw{};
  }
};

template <class T>
hipError_t upload(T** d, const T* h, size_t n) {
  hipError_t e = hipMalloc((void**)d, std::max<size_t>(n, 1) * sizeof(T));
  if (e != hipSuccess) return e;
  if (n) e = hipMemcpy(*d, h, n * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

void free_ctx(rtbte_ctx* c) {
  if (!c) return;
  void* ps[] = {c->ch, c->groups, c->items, c->order, c->item_ptr, c->row_group, c->partial_items,
                c->mix_idx, c->mix_wq, c->mix_scale, c->popf, c->pk, c->pkw, c->row_inst, c->info_d, c->st,
                c->st_fast, c->st_slow, c->mra, c->mis_keep, c->energy_d,
                c->kbuf[0], c->kbuf[1], c->kbuf[2], c->kbuf[3], c->kbuf[4], c->zb[0], c->zb[1],
                c->ynew, c->lte, c->tmp, c->tmp2, c->fs[0], c->fs[1], c->fs[2], c->forcing,
                c->partial, c->tvec, c->summary_d, c->tblocks, c->border, c->tiles, c->bnd, c->ppm, c->health};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  for (auto& g : c->graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.g);
  }
  if (c->cap) (void)hipStreamDestroy(c->cap);
  for (auto& p : c->pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  for (auto& p : c->pool) { (void)hipEventDestroy(p.first); (void)hipEventDestroy(p.second); }
  if (c->summary_h) (void)hipHostFree(c->summary_h);
  if (c->scal_h) (void)hipHostFree(c->scal_h);
  delete c;
}

bool valid_group_rows(int g) { return g == 1 || g == 2 || g == 4 || g == 8 || g == 12 || g == 16; }

// Default channels per work item: about 40k items, within [2048, 65536].
int64_t auto_item_channels(int64_t n_ch) { return std::min<int64_t>(65536, std::max<int64_t>(2048, n_ch / 40960)); }

// (Re)build the work items: each group's channels cut into near-equal pieces
// of at most `ich` channels; processing order longest first (stable).
hipError_t build_items(rtbte_ctx* c, int64_t ich) {
  if (ich <= 0) ich = auto_item_channels(c->n_ch);
  void* old[] = {c->items, c->order, c->item_ptr, c->partial_items};
  for (void* p : old)
    if (p) (void)hipFree(p);
  c->items = nullptr; c->order = nullptr; c->item_ptr = nullptr; c->partial_items = nullptr;
  c->item_channels = ich;
  std::vector<Item> items;
  std::vector<int64_t> iptr((size_t)c->n_groups + 1, 0);
  for (int64_t gi = 0; gi < c->n_groups; ++gi) {
    const Group& gr = c->groups_h[gi];
    const int64_t len = gr.end - gr.start;
    const int64_t n = len ? (len + ich - 1) / ich : 0;
    for (int64_t q = 0; q < n; ++q) {
      Item it{};
      it.lo = gr.start + len * q / n;
      it.hi = gr.start + len * (q + 1) / n;
      it.group = (int32_t)gi;
      items.push_back(it);
    }
    iptr[gi + 1] = (int64_t)items.size();
  }
  c->n_items = (int64_t)items.size();
  std::vector<int32_t> order((size_t)c->n_items);
  for (int64_t i = 0; i < c->n_items; ++i) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    return items[x].hi - items[x].lo > items[y].hi - items[y].lo;
  });
  hipError_t e = upload(&c->items, items.data(), items.size());
  if (e == hipSuccess) e = upload(&c->order, order.data(), order.size());
  if (e == hipSuccess) e = upload(&c->item_ptr, iptr.data(), iptr.size());
  if (e == hipSuccess)
    c->partial_items = dalloc<double>((size_t)std::max<int64_t>(c->n_items, 1) * kMaxGroupRows, &e);
  for (auto& g : c->graphs) {  // captured launches hold the old tables
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.g);
  }
  c->graphs.clear();
  return e;
}

// Tiled launch (packed layouts): the channels of every group segment cut at
// key-block bounds, sets of kTileWaves consecutive segments of one kind of
// one instance, the other-partner window of each (set, key block), and
// blocks that run a set through a range of key blocks of about
// kTileWaves * ich channels, each wavefront writing one item.  Items are
// stored group by group (the row kernel sums a group's items in order).
hipError_t build_tiles(rtbte_ctx* c, int64_t ich) {
  const bool mixed = c->mixed;
  const uint64_t* words = mixed ? reinterpret_cast<const uint64_t*>(c->mix_idx) : c->pk;
  if (!words) return hipErrorInvalidValue;
  const int64_t KL = mixed ? kTileKey32 : kTileKey64;
  const int64_t OC = mixed ? kTileOther32 : kTileOther64;
  if (ich <= 0) ich = auto_item_channels(c->n_ch);
  c->item_channels = ich;
  void* old[] = {c->items, c->order, c->item_ptr, c->partial_items, c->tblocks, c->border, c->tiles, c->bnd};
  for (void* p : old)
    if (p) (void)hipFree(p);
  c->items = nullptr; c->order = nullptr; c->item_ptr = nullptr; c->partial_items = nullptr;
  c->tblocks = nullptr; c->border = nullptr; c->tiles = nullptr; c->bnd = nullptr;
  c->n_items = c->n_blocks = 0;
  c->tiled = false;
  c->tile_in_window = 0.0;
  // 1. segments and the offsets of their bounds
  struct SegH { int32_t group, kind, inst, n_kb; int64_t lo, hi, off; };
  std::vector<SegH> sh;
  std::vector<SegRange> sr;
  int64_t nbnd = 0;
  for (int64_t gi = 0; gi < c->n_groups; ++gi) {
    const Group& g = c->groups_h[gi];
    const InstInfo& in = c->info[g.inst];
    const int32_t n_kb = (int32_t)(((int64_t)in.n_el + in.n_ph + KL - 1) / KL);
    auto add = [&](int64_t lo, int64_t hi, int32_t kind) {
      sh.push_back({(int32_t)gi, kind, g.inst, n_kb, lo, hi, nbnd});
      sr.push_back({lo, hi, nbnd, kind, n_kb});
      nbnd += n_kb + 1;
    };
    if (!g.phonon) add(g.start, g.end, 0);
    else {
      add(g.start, g.split, 1);
      add(g.split, g.end, 2);
    }
  }
  // 2. key-block bounds (device), copied back
  SegRange* sr_d = nullptr;
  hipError_t e = upload(&sr_d, sr.data(), sr.size());
  if (e == hipSuccess) c->bnd = dalloc<int64_t>((size_t)std::max<int64_t>(nbnd, 1), &e);
  if (e == hipSuccess) e = launch_key_bounds(words, c->pack_p, sr_d, (int64_t)sr.size(), KL, c->bnd, 0);
  std::vector<int64_t> bnd((size_t)nbnd);
  if (e == hipSuccess && nbnd) e = hipMemcpy(bnd.data(), c->bnd, (size_t)nbnd * sizeof(int64_t), hipMemcpyDeviceToHost);
  if (sr_d) (void)hipFree(sr_d);
  if (e != hipSuccess) return e;
  // 3. sets: consecutive segments of one kind of one instance
  std::vector<std::vector<int32_t>> sets;   // segment indices
  for (int kind = 0; kind < 3; ++kind) {
    std::vector<int32_t> cur;
    int32_t inst = -1;
    for (int32_t si = 0; si < (int32_t)sh.size(); ++si) {
      if (sh[si].kind != kind) continue;
      if (sh[si].inst != inst || (int)cur.size() == kTileWaves) {
        if (!cur.empty()) sets.push_back(cur);
        cur.clear();
        inst = sh[si].inst;
      }
      cur.push_back(si);
    }
    if (!cur.empty()) sets.push_back(cur);
  }
  // 4. the other-partner span of every non-empty (set, key block)
  std::vector<SpanJob> jobs;
  std::vector<int64_t> tile_of;     // per set: first tile index; tiles are [set][j]
  std::vector<int64_t> job_tile;    // tile index of each job
  int64_t ntiles = 0;
  for (const auto& st : sets) {
    tile_of.push_back(ntiles);
    const int32_t n_kb = sh[st[0]].n_kb;
    for (int32_t j = 0; j < n_kb; ++j) {
      int64_t tot = 0;
      SpanJob jb{};
      for (int w = 0; w < kTileWaves; ++w) jb.bndo[w] = -1;
      for (size_t w = 0; w < st.size(); ++w) {
        const SegH& s = sh[st[w]];
        tot += bnd[s.off + j + 1] - bnd[s.off + j];
        jb.bndo[w] = s.off;
      }
      if (tot > 0) {
        jb.j = j;
        jb.kind = sh[st[0]].kind;
        jobs.push_back(jb);
        job_tile.push_back(ntiles + j);
      }
    }
    ntiles += n_kb;
  }
  std::vector<Tile> tiles((size_t)std::max<int64_t>(ntiles, 1), Tile{kTileEmpty, 0u});
  if (!jobs.empty()) {
    SpanJob* jobs_d = nullptr;
    uint32_t* span_d = nullptr;
    e = upload(&jobs_d, jobs.data(), jobs.size());
    if (e == hipSuccess) span_d = dalloc<uint32_t>(2 * jobs.size(), &e);
    if (e == hipSuccess) e = launch_tile_span(words, c->pack_p, jobs_d, (int64_t)jobs.size(), c->bnd, span_d, 0);
    std::vector<uint32_t> span(2 * jobs.size());
    if (e == hipSuccess) e = hipMemcpy(span.data(), span_d, span.size() * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (jobs_d) (void)hipFree(jobs_d);
    if (span_d) (void)hipFree(span_d);
    if (e != hipSuccess) return e;
    // a tile whose other partners do not fit the window stages none of them
    // (its gathers of the other partner all go to global memory)
    for (size_t k = 0; k < jobs.size(); ++k) {
      const uint32_t mn = span[2 * k], mx = span[2 * k + 1];
      const int64_t len = (int64_t)mx - mn + 1;
      tiles[(size_t)job_tile[k]] = len <= OC ? Tile{mn, (uint32_t)len} : Tile{mn, 0u};
      c->tile_in_window += len <= OC ? 1.0 : 0.0;
    }
    c->tile_in_window /= (double)jobs.size();
  }
  // 5. blocks: each set through ranges of key blocks of about kTileWaves * ich channels
  struct ItemH { int32_t group; int64_t lo, hi; int32_t block, wave; };
  std::vector<ItemH> ih;
  std::vector<TileBlock> blocks;
  std::vector<int64_t> work;        // the longest wavefront range of each block
  const int64_t target = (int64_t)kTileWaves * ich;
  for (size_t si = 0; si < sets.size(); ++si) {
    const auto& st = sets[si];
    const int32_t n_kb = sh[st[0]].n_kb;
    int32_t j0 = 0;
    while (j0 < n_kb) {
      int64_t tot = 0;
      int32_t j1 = j0;
      while (j1 < n_kb && (tot == 0 || tot < target)) {
        for (int32_t s : st) tot += bnd[sh[s].off + j1 + 1] - bnd[sh[s].off + j1];
        ++j1;
      }
      if (tot > 0) {
        TileBlock b{};
        for (int w = 0; w < kTileWaves; ++w) { b.bndo[w] = -1; b.item[w] = -1; }
        b.inst = sh[st[0]].inst;
        b.kind = sh[st[0]].kind;
        b.j0 = j0;
        b.j1 = j1;
        b.tile0 = (int32_t)(tile_of[si] + j0);
        int64_t mx = 0;
        for (size_t w = 0; w < st.size(); ++w) {
          const SegH& s = sh[st[w]];
          const int64_t lo = bnd[s.off + j0], hi = bnd[s.off + j1];
          b.bndo[w] = s.off;
          if (hi > lo) ih.push_back({s.group, lo, hi, (int32_t)blocks.size(), (int32_t)w});
          mx = std::max(mx, hi - lo);
        }
        blocks.push_back(b);
        work.push_back(mx);
      }
      j0 = j1;
    }
  }
  // 6. items group by group (stable), and each block's wave items
  std::vector<int32_t> iord(ih.size());
  for (size_t k = 0; k < ih.size(); ++k) iord[k] = (int32_t)k;
  std::stable_sort(iord.begin(), iord.end(), [&](int32_t x, int32_t y) { return ih[x].group < ih[y].group; });
  std::vector<Item> items(ih.size());
  std::vector<int64_t> iptr((size_t)c->n_groups + 1, 0);
  for (size_t k = 0; k < iord.size(); ++k) {
    const ItemH& x = ih[iord[k]];
    items[k] = Item{x.lo, x.hi, x.group, 0};
    blocks[(size_t)x.block].item[x.wave] = (int32_t)k;
    iptr[(size_t)x.group + 1]++;
  }
  for (int64_t gi = 0; gi < c->n_groups; ++gi) iptr[gi + 1] += iptr[gi];
  c->n_items = (int64_t)items.size();
  c->n_blocks = (int64_t)blocks.size();
  std::vector<int32_t> order((size_t)c->n_items), border((size_t)c->n_blocks);
  for (int64_t i = 0; i < c->n_items; ++i) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    return items[x].hi - items[x].lo > items[y].hi - items[y].lo;
  });
  for (int64_t i = 0; i < c->n_blocks; ++i) border[i] = (int32_t)i;
  std::stable_sort(border.begin(), border.end(), [&](int32_t x, int32_t y) { return work[x] > work[y]; });
  e = upload(&c->items, items.data(), items.size());
  if (e == hipSuccess) e = upload(&c->order, order.data(), order.size());
  if (e == hipSuccess) e = upload(&c->item_ptr, iptr.data(), iptr.size());
  if (e == hipSuccess)
    c->partial_items = dalloc<double>((size_t)std::max<int64_t>(c->n_items, 1) * kMaxGroupRows, &e);
  if (e == hipSuccess) e = upload(&c->tblocks, blocks.data(), blocks.size());
  if (e == hipSuccess) e = upload(&c->border, border.data(), border.size());
  if (e == hipSuccess) e = upload(&c->tiles, tiles.data(), tiles.size());
  if (e != hipSuccess) return e;
  c->tiled = true;
  for (auto& g : c->graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.g);
  }
  c->graphs.clear();
  return hipSuccess;
}

// Work items of the context's launch mode: tiled when it was built tiled.
hipError_t rebuild_items(rtbte_ctx* c, int64_t ich) {
  return c->tiled ? build_tiles(c, ich) : build_items(c, ich);
}

}  // namespace

// Build a context with the launch shape in `opts` (no tuning).
namespace {

inline uint64_t mix64(uint64_t z) {   // splitmix64 finaliser (Steele, Lea, Flood, OOPSLA'14)
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Is every ph-ph entry (l; a, b) with a != b matched by (l; b, a) with the
// same |V3|^2, as in the sum over ordered partner pairs?  Compared as equal
// multisets through counts and wrapping sums of a 64-bit mix of (l, min,
// max, |V3|^2 bits) over the a < b and the a > b entries.  *folded receives
// the number of emission channels the a > b entries would give (they are
// carried by their mirrors when the list is folded).
bool pp_mirror_symmetric(const rtbte_problem& p, int64_t* folded) {
  uint64_t s_lt = 0, s_gt = 0;
  int64_t n_lt = 0, n_gt = 0, nf = 0;
  const double cut = p.nsigma * p.sigma_pp;
#pragma omp parallel for reduction(+ : s_lt, s_gt, n_lt, n_gt, nf) schedule(static)
  for (int64_t e = 0; e < p.n_pp; ++e) {
    const int32_t l = p.pp_row[e], a = p.pp_a[e], b = p.pp_b[e];
    if (a == b) continue;
    uint64_t vb = 0;   // no values (matrix-free weights): the model is symmetric
    if (p.pp_v2) std::memcpy(&vb, &p.pp_v2[e], sizeof vb);
    const uint64_t h = mix64(mix64(mix64((uint64_t)(uint32_t)l + 0x9E3779B97F4A7C15ull) +
                                   (uint64_t)(uint32_t)std::min(a, b)) +
                             (uint64_t)(uint32_t)std::max(a, b)) + mix64(vb ^ 0xD1B54A32D192ED03ull);
    if (a < b) {
      s_lt += h;
      ++n_lt;
    } else {
      s_gt += h;
      ++n_gt;
      // the emission channel of this entry, kept as the preparation keeps it
      const double w = p.hw[l], wa = p.hw[a], wb = p.hw[b];
      if (!(w < p.hw_cut || wa < p.hw_cut || wb < p.hw_cut) && std::fabs(-w + wa + wb) <= cut) ++nf;
    }
  }
  *folded = nf;
  return n_lt > 0 && s_lt == s_gt && n_lt == n_gt;
}

}  // namespace

static int create_impl(const rtbte_problem* problems, int32_t n_inst, const rtbte_options* opts,
                       rtbte_ctx** out) {
  if (!out) return fail(nullptr, RTBTE_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!problems || n_inst < 1) return fail(nullptr, RTBTE_E_INVAL, "need n_inst >= 1 problems");
  rtbte_options o;
  if (opts) o = *opts;
  else rtbte_default_options(&o);
  if (o.precision != RTBTE_FP64 && o.precision != RTBTE_MIXED)
    return fail(nullptr, RTBTE_E_INVAL, "precision must be RTBTE_FP64 or RTBTE_MIXED");
  if (o.fp64_layout < RTBTE_F64_AUTO || o.fp64_layout > RTBTE_F64_PLAIN)
    return fail(nullptr, RTBTE_E_INVAL, "fp64_layout must be RTBTE_F64_AUTO, RTBTE_F64_PACKED or RTBTE_F64_PLAIN");
  if (o.mixed_weights < RTBTE_W_AUTO || o.mixed_weights > RTBTE_W_BF16_EPH)
    return fail(nullptr, RTBTE_E_INVAL, "mixed_weights must be one of RTBTE_W_AUTO .. RTBTE_W_BF16_EPH");
  if (o.group_rows_el == 0) o.group_rows_el = 8;
  if (o.group_rows_ph == 0) o.group_rows_ph = 16;
  if (!valid_group_rows(o.group_rows_el) || !valid_group_rows(o.group_rows_ph))
    return fail(nullptr, RTBTE_E_INVAL, "group_rows_el / group_rows_ph must be 0, 1, 2, 4, 8, 12 or 16");
  if (o.item_channels < 0) return fail(nullptr, RTBTE_E_INVAL, "item_channels must be >= 0");
  if (o.fp64_check < 0) return fail(nullptr, RTBTE_E_INVAL, "fp64_check must be >= 0");
  if (o.pp_fold != 0 && o.pp_fold != 1) return fail(nullptr, RTBTE_E_INVAL, "pp_fold must be 0 or 1");
  if (o.small_nef < 1 || !(o.eta_fail_repeat > 0.0))
    return fail(nullptr, RTBTE_E_INVAL, "small_nef must be >= 1 and eta_fail_repeat > 0");
  if (!(o.rtol >= 0) || !(o.atol_el >= 0) || !(o.atol_ph >= 0) || o.pid_order <= 0 ||
      o.steps_per_poll < 1 || o.max_fails < 0)
    return fail(nullptr, RTBTE_E_INVAL, "invalid tolerances or controller options");
  for (int i = 0; i < n_inst; ++i) {
    int rc = check_problem(problems[i], i, o.pp_model != nullptr);
    if (rc) return rc;
  }
  if (o.pp_model) {
    if (o.tiled) return fail(nullptr, RTBTE_E_UNSUPPORTED, "matrix-free ph-ph weights need tiled = 0");
    for (int i = 0; i < n_inst; ++i) {
      const rtbte_pp_model& m = o.pp_model[i];
      int64_t nq = m.L;
      for (int d = 1; d < m.dim; ++d) nq *= m.L;
      if ((m.dim != 2 && m.dim != 3) || m.L < 1 || m.n_modes < 1 || nq * m.n_modes != problems[i].n_ph ||
          !std::isfinite(m.ln_mu) || !std::isfinite(m.ln_sigma))
        return fail(nullptr, RTBTE_E_INVAL, "instance %d: pp_model does not describe its %d phonon states", i,
                    problems[i].n_ph);
    }
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(nullptr, RTBTE_E_HIP, "no HIP device available");
  if (o.device < 0 || o.device >= ndev) return fail(nullptr, RTBTE_E_INVAL, "device %d out of range", o.device);
  if (hipSetDevice(o.device) != hipSuccess) return fail(nullptr, RTBTE_E_HIP, "hipSetDevice failed");

  void* scratch_dev = nullptr;
  {
    const hipError_t e = scratch_setup(o.device, &scratch_dev);
    if (e != hipSuccess)
      return fail(nullptr, RTBTE_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  }

  const int GE = o.group_rows_el, GP = o.group_rows_ph;
  rtbte_ctx* c = new rtbte_ctx();
  c->device = o.device;
  c->scratch_dev = scratch_dev;
  c->opt = o;
  c->n_inst = n_inst;
  c->info.resize(n_inst);
  int64_t off = 0;
  for (int i = 0; i < n_inst; ++i) {
    c->info[i].off = off;
    c->info[i].n_el = problems[i].n_el;
    c->info[i].n_ph = problems[i].n_ph;
    off += (int64_t)problems[i].n_el + problems[i].n_ph;
  }
  c->ny = off;
  c->energy_h.resize((size_t)off);
  for (int i = 0; i < n_inst; ++i) {
    const rtbte_problem& p = problems[i];
    if ((p.n_el > 0 && !p.eps) || (p.n_ph > 0 && !p.hw)) continue;   // check_problem rejected it already
    std::copy(p.eps, p.eps + p.n_el, c->energy_h.begin() + c->info[i].off);
    std::copy(p.hw, p.hw + p.n_ph, c->energy_h.begin() + c->info[i].off + p.n_el);
  }
  if (c->ny > (int64_t)kPosMask) {
    free_ctx(c);
    return fail(nullptr, RTBTE_E_INVAL, "state vector too long (%lld > %d)", (long long)off, kPosMask);
  }
  int64_t big = 1;   // largest instance; its positions need P bits
  for (int i = 0; i < n_inst; ++i) big = std::max<int64_t>(big, (int64_t)problems[i].n_el + problems[i].n_ph);
  int P = 1;
  while (((int64_t)1 << P) < big) ++P;
  if (o.precision == RTBTE_FP64) {
    // packed 12-byte channels need P <= 19 (M = min(80 - 2P, 52) >= 42 mantissa bits)
    if (o.fp64_layout == RTBTE_F64_PACKED && P > 19) {
      free_ctx(c);
      return fail(nullptr, RTBTE_E_INVAL, "RTBTE_F64_PACKED needs instances of at most 2^19 states (%lld given)",
                  (long long)big);
    }
    const bool pk = o.fp64_layout == RTBTE_F64_PACKED || (o.fp64_layout == RTBTE_F64_AUTO && P <= 19);
    c->wfmt = pk ? -2 : -1;
    c->pack_p = pk ? P : 0;
    c->pack_m = pk ? std::min(80 - 2 * P, 52) : 0;
    c->f64_m = c->pack_m;
  }
  if (o.precision == RTBTE_MIXED) {
    // weight format: the packed 8-byte words need P-bit positions relative to
    // the instance with P <= 20 (mantissa M = min(53 - 2P, 23) >= 13 bits)
    int w = o.mixed_weights;
    if (w == RTBTE_W_AUTO) w = P <= 20 ? RTBTE_W_PACK8 : RTBTE_W_F16X;
    if (w == RTBTE_W_PACK8 && P > 20) {
      free_ctx(c);
      return fail(nullptr, RTBTE_E_INVAL, "RTBTE_W_PACK8 needs instances of at most 2^20 states (%lld given)",
                  (long long)big);
    }
    if (w != RTBTE_W_PACK8 && c->ny > (int64_t)kMixPosMask + 1) {
      free_ctx(c);
      return fail(nullptr, RTBTE_E_INVAL, "the 10-byte mixed formats hold at most %d states (%lld given)",
                  kMixPosMask + 1, (long long)off);
    }
    c->wfmt = w;
    c->pack_p = P;
    c->pack_m = std::min(53 - 2 * P, 23);   // at most FP32's 23 mantissa bits; spare high bits stay 0
    // FP64 lists kept for the mixed-vs-FP64 check: packed when P <= 19 (the
    // FP64 default), else the plain 16-byte channels
    c->keep64 = o.fp64_check > 0;
    c->f64_m = c->keep64 && P <= 19 ? std::min(80 - 2 * P, 52) : 0;
  }
  c->err64.assign((size_t)n_inst, -1.0);
  c->folded.assign((size_t)n_inst, 0);
  c->counts.assign(3 * (size_t)n_inst, 0);

  // Pass 1: upload raw entries and count kept channels per destination group.
  std::vector<DevRaw> raws((size_t)n_inst);
  std::vector<std::vector<int64_t>> cnt_e(n_inst), cnt_pe(n_inst), cnt_pp(n_inst);
  auto cleanup = [&](int code) {
    for (auto& r : raws) r.release();
    std::string msg = c->err;
    free_ctx(c);
    if (!msg.empty()) g_create_error = msg;
    return code;
  };
  std::vector<PrepArgs> pe(n_inst), ppe(n_inst), ppp(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    const rtbte_problem& p = problems[i];
    DevRaw& d = raws[i];
    std::vector<int64_t> perm, gptr;
    hipError_t e = hipSuccess;
#define UP(dst, src, n)                                                             \
  do {                                                                              \
    e = upload(&(dst), (src), (size_t)(n));                                         \
    if (e != hipSuccess) {                                                          \
      fail(c, e == hipErrorOutOfMemory ? RTBTE_E_NOMEM : RTBTE_E_HIP, "upload: %s", \
           hipGetErrorString(e));                                                   \
      return cleanup(e == hipErrorOutOfMemory ? RTBTE_E_NOMEM : RTBTE_E_HIP);       \
    }                                                                               \
  } while (0)
    UP(d.eps, p.eps, p.n_el);
    UP(d.hw, p.hw, p.n_ph);
    UP(d.er, p.eph_row, p.n_eph);
    UP(d.es, p.eph_partner, p.n_eph);
    UP(d.ep, p.eph_phonon, p.n_eph);
    UP(d.eg, p.eph_g2, p.n_eph);
    UP(d.pr, p.pp_row, p.n_pp);
    UP(d.pa, p.pp_a, p.n_pp);
    UP(d.pb, p.pp_b, p.n_pp);
    if (p.pp_v2) UP(d.pv, p.pp_v2, p.n_pp);   // absent with matrix-free weights (values taken as 1)
    // electron side: groups of electron rows, merged by phonon (the shared q)
    group_entries(p.n_eph, p.eph_row, p.n_el, GE, p.eph_phonon, perm, gptr);
    if (!perm.empty()) UP(d.perm_e, perm.data(), perm.size());
    UP(d.ptr_e, gptr.data(), gptr.size());
    // phonon side of e-ph: groups of phonon rows, merged by the initial electron
    group_entries(p.n_eph, p.eph_phonon, p.n_ph, GP, p.eph_row, perm, gptr);
    if (!perm.empty()) UP(d.perm_pe, perm.data(), perm.size());
    UP(d.ptr_pe, gptr.data(), gptr.size());
    // ph-ph: groups of phonon rows, merged by the first partner
    group_entries(p.n_pp, p.pp_row, p.n_ph, GP, p.pp_a, perm, gptr);
    if (!perm.empty()) UP(d.perm_pp, perm.data(), perm.size());
    UP(d.ptr_pp, gptr.data(), gptr.size());
#undef UP
    const int32_t nge = (p.n_el + GE - 1) / GE, ngp = (p.n_ph + GP - 1) / GP;
    d.cnt_e = dalloc<int64_t>(nge, &e);
    if (e == hipSuccess) d.cnt_pe = dalloc<int64_t>(ngp, &e);
    if (e == hipSuccess) d.cnt_pp = dalloc<int64_t>(ngp, &e);
    if (e != hipSuccess) {
      fail(c, RTBTE_E_NOMEM, "count buffers: %s", hipGetErrorString(e));
      return cleanup(RTBTE_E_NOMEM);
    }
    const bool fold = o.pp_fold && pp_mirror_symmetric(p, &c->folded[(size_t)i]);
    if (!fold) c->folded[(size_t)i] = 0;
    const double pre_el = (2.0 * kPi / kHbarEvFs) / (double)p.n_q_total;
    const double pre_ph = (4.0 * kPi / kHbarEvFs) / (double)p.n_k_total;
    const double pre_pp = (36.0 * kPi / kHbarEvFs) / (double)p.n_q_total;
    PrepArgs a{};
    a.eps = d.eps;
    a.hw = d.hw;
    a.y_off = c->info[i].off;
    a.n_el = p.n_el;
    a.hw_cut = p.hw_cut;
    a.group_rows = GE;
    // e-ph electron side
    a.row = d.er; a.i0 = d.es; a.i1 = d.ep; a.val = d.eg; a.perm = d.perm_e; a.raw_ptr = d.ptr_e;
    a.n_dest = nge; a.sigma = p.sigma_eph; a.cut = p.nsigma * p.sigma_eph; a.pre = pre_el;
    a.pre2 = pre_el; a.kind = 0; a.count = d.cnt_e;
    pe[i] = a;
    // ph-e
    a.group_rows = GP;
    a.perm = d.perm_pe; a.raw_ptr = d.ptr_pe; a.n_dest = ngp; a.pre = pre_ph; a.pre2 = pre_ph;
    a.kind = 1; a.count = d.cnt_pe;
    ppe[i] = a;
    // ph-ph
    a.row = d.pr; a.i0 = d.pa; a.i1 = d.pb; a.val = d.pv; a.perm = d.perm_pp; a.raw_ptr = d.ptr_pp;
    a.n_dest = ngp; a.sigma = p.sigma_pp; a.cut = p.nsigma * p.sigma_pp; a.pre = pre_pp;
    a.pre2 = 2.0 * pre_pp; a.kind = 2; a.count = d.cnt_pp; a.fold_em = fold ? 1 : 0;
    ppp[i] = a;
    e = launch_prep_count(pe[i], 0);
    if (e == hipSuccess) e = launch_prep_count(ppe[i], 0);
    if (e == hipSuccess) e = launch_prep_count(ppp[i], 0);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    cnt_e[i].resize(nge);
    cnt_pe[i].resize(ngp);
    cnt_pp[i].resize(ngp);
    if (e == hipSuccess && nge) e = hipMemcpy(cnt_e[i].data(), d.cnt_e, nge * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && ngp) e = hipMemcpy(cnt_pe[i].data(), d.cnt_pe, ngp * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && ngp) e = hipMemcpy(cnt_pp[i].data(), d.cnt_pp, ngp * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      fail(c, RTBTE_E_HIP, "channel count: %s", hipGetErrorString(e));
      return cleanup(RTBTE_E_HIP);
    }
  }

  // Group table over the concatenated state vector.
  std::vector<Group> groups;
  std::vector<int64_t> glen;
  std::vector<std::vector<int64_t>> base_e(n_inst), base_pe(n_inst), base_pp(n_inst);
  {
    int64_t pos = 0;
    for (int i = 0; i < n_inst; ++i) {
      // every instance starts on a 512-channel boundary (the slots between
      // instances hold zeros and are only read by masked-off lanes), so
      // mixed-precision scale blocks and the 256-channel tiles of the FP64
      // packed stream never straddle two instances: an instance is stored,
      // and computes, exactly as it would alone
      pos = (pos + kMixBlock - 1) / kMixBlock * kMixBlock;
      const InstInfo& in = c->info[i];
      const int32_t nge = (int32_t)cnt_e[i].size(), ngp = (int32_t)cnt_pe[i].size();
      base_e[i].resize(nge);
      base_pe[i].resize(ngp);
      base_pp[i].resize(ngp);
      for (int32_t g = 0; g < nge; ++g) {
        Group gr{};
        gr.start = pos;
        base_e[i][g] = pos;
        pos += cnt_e[i][g];
        gr.split = gr.end = pos;
        gr.row0 = (int32_t)(in.off + (int64_t)g * GE);
        gr.inst = i;
        gr.nrows = std::min(GE, in.n_el - g * GE);
        gr.phonon = 0;
        groups.push_back(gr);
        glen.push_back(cnt_e[i][g]);
        c->counts[3 * i] += cnt_e[i][g];
      }
      for (int32_t g = 0; g < ngp; ++g) {
        Group gr{};
        gr.start = pos;
        base_pe[i][g] = pos;
        pos += cnt_pe[i][g];
        gr.split = pos;
        base_pp[i][g] = pos;
        pos += cnt_pp[i][g];
        gr.end = pos;
        gr.row0 = (int32_t)(in.off + in.n_el + (int64_t)g * GP);
        gr.inst = i;
        gr.nrows = std::min(GP, in.n_ph - g * GP);
        gr.phonon = 1;
        groups.push_back(gr);
        glen.push_back(cnt_pe[i][g] + cnt_pp[i][g]);
        c->counts[3 * i + 1] += cnt_pe[i][g];
        c->counts[3 * i + 2] += cnt_pp[i][g];
      }
    }
    c->n_ch = pos;
    c->n_groups = (int64_t)groups.size();
  }
  hipError_t e = hipSuccess;
  c->ch = dalloc<Channel>((size_t)c->n_ch, &e);
  if (e != hipSuccess) {
    fail(c, RTBTE_E_NOMEM, "channel lists (%lld channels): %s", (long long)c->n_ch, hipGetErrorString(e));
    return cleanup(RTBTE_E_NOMEM);
  }
  // Unwritten slots would never be read, but keep them harmless (index 0, weight 0).
  e = hipMemset(c->ch, 0, (size_t)std::max<int64_t>(c->n_ch, 1) * sizeof(Channel));
  if (e != hipSuccess) {
    fail(c, RTBTE_E_HIP, "channel clear: %s", hipGetErrorString(e));
    return cleanup(RTBTE_E_HIP);
  }
  // Pass 2: write the channels.
  for (int i = 0; i < n_inst; ++i) {
    DevRaw& d = raws[i];
    e = upload(&d.base_e, base_e[i].data(), base_e[i].size());
    if (e == hipSuccess) e = upload(&d.base_pe, base_pe[i].data(), base_pe[i].size());
    if (e == hipSuccess) e = upload(&d.base_pp, base_pp[i].data(), base_pp[i].size());
    pe[i].base = d.base_e; pe[i].out = c->ch;
    ppe[i].base = d.base_pe; ppe[i].out = c->ch;
    ppp[i].base = d.base_pp; ppp[i].out = c->ch;
    if (e == hipSuccess) e = launch_prep_fill(pe[i], 0);
    if (e == hipSuccess) e = launch_prep_fill(ppe[i], 0);
    if (e == hipSuccess) e = launch_prep_fill(ppp[i], 0);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      fail(c, RTBTE_E_HIP, "channel fill: %s", hipGetErrorString(e));
      return cleanup(RTBTE_E_HIP);
    }
    d.release();
  }

  std::vector<int32_t> rgroup((size_t)c->ny, 0);
  for (int64_t gi = 0; gi < c->n_groups; ++gi)
    for (int32_t j = 0; j < groups[gi].nrows; ++j) rgroup[(size_t)groups[gi].row0 + j] = (int32_t)gi;
  e = upload(&c->groups, groups.data(), groups.size());
  if (e == hipSuccess) e = upload(&c->row_group, rgroup.data(), rgroup.size());
  c->groups_h = std::move(groups);
  if (e == hipSuccess) e = build_items(c, o.item_channels);
  if (e == hipSuccess) e = upload(&c->info_d, c->info.data(), c->info.size());
  if (e == hipSuccess && c->ny > 0) e = upload(&c->energy_d, c->energy_h.data(), c->energy_h.size());
  if (e == hipSuccess && o.precision == RTBTE_MIXED) {
    // compact weights with per-block FP32 scales; the FP64 channels are freed
    const bool pack = c->wfmt == RTBTE_W_PACK8;
    const int64_t nblk = (c->n_ch + kMixBlock - 1) / kMixBlock;
    c->mix_scale = dalloc<float>((size_t)std::max<int64_t>(nblk, 1), &e);
    if (e == hipSuccess) c->mix_idx = dalloc<int2>((size_t)c->n_ch + 4, &e);
    if (e == hipSuccess && !pack) c->mix_wq = dalloc<uint16_t>((size_t)c->n_ch + 8, &e);
    if (e == hipSuccess) c->popf = dalloc<float>((size_t)c->ny, &e);
    if (e == hipSuccess) e = hipMemset(c->mix_idx, 0, ((size_t)c->n_ch + 4) * sizeof(int2));
    if (e == hipSuccess && !pack) e = hipMemset(c->mix_wq, 0, ((size_t)c->n_ch + 8) * sizeof(uint16_t));
    if (e == hipSuccess) e = launch_mix_scales(c->ch, c->n_ch, pack ? 1.0f : 0x1p-15f, c->mix_scale, 0);
    if (e == hipSuccess && pack)
      e = launch_mix_pack8(c->ch, c->n_ch, c->groups, c->n_groups, c->info_d, c->mix_scale, c->pack_p,
                           c->pack_m, c->mix_idx, 0);
    if (e == hipSuccess && !pack)
      e = launch_mix_convert(c->ch, c->n_ch, c->groups, c->n_groups, c->mix_scale, c->wfmt, c->mix_idx,
                             c->mix_wq, 0);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess && !c->keep64) {
      e = hipFree(c->ch);
      c->ch = nullptr;
    }
    c->mixed = true;
  }
  if (e == hipSuccess && (c->mixed ? c->f64_m > 0 : c->wfmt == -2)) {
    // FP64 packed channels; the 16-byte channels are freed
    c->pk = dalloc<uint64_t>((size_t)c->n_ch + 2, &e);
    // low weight words: whole 256-channel tiles (read a tile at a time)
    const size_t nw = ((size_t)c->n_ch + 255) / 256 * 256 + 256;
    if (e == hipSuccess) c->pkw = dalloc<uint32_t>(nw, &e);
    if (e == hipSuccess) e = hipMemset(c->pk, 0, ((size_t)c->n_ch + 2) * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMemset(c->pkw, 0, nw * sizeof(uint32_t));
    if (e == hipSuccess)
      e = launch_pack12(c->ch, c->n_ch, c->groups, c->n_groups, c->info_d, c->pack_p, c->f64_m, c->pk, c->pkw, 0);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) {
      e = hipFree(c->ch);
      c->ch = nullptr;
    }
  }
  // tiled launch blocks over the packed words
  if (e == hipSuccess && o.tiled && (c->mixed ? c->wfmt == RTBTE_W_PACK8 : c->pk != nullptr))
    e = build_tiles(c, o.item_channels);
  // matrix-free ph-ph weights: the models with each instance's prefactor,
  // width, fold and phonon offset (packed words only)
  if (e == hipSuccess && o.pp_model) {
    if (c->mixed ? c->wfmt != RTBTE_W_PACK8 : c->pk == nullptr) {
      free_ctx(c);
      return fail(nullptr, RTBTE_E_UNSUPPORTED,
                  "matrix-free ph-ph weights need packed channels (FP64 packed or RTBTE_W_PACK8)");
    }
    std::vector<PpModel> pm((size_t)n_inst);
    for (int i = 0; i < n_inst; ++i) {
      const rtbte_pp_model& m = o.pp_model[i];
      PpModel& q = pm[(size_t)i];
      q.dim = m.dim;
      q.L = m.L;
      q.n_modes = m.n_modes;
      q.folded = c->folded[(size_t)i] > 0 ? 1 : 0;
      q.key0 = m.key0;
      q.key1 = m.key1;
      q.stream = m.stream;
      q.n_el = (uint32_t)problems[i].n_el;
      q.ln_mu = m.ln_mu;
      q.ln_sigma = m.ln_sigma;
      const double pre = (36.0 * kPi / kHbarEvFs) / (double)problems[i].n_q_total;
      q.pre_norm = pre / (problems[i].sigma_pp * kSqrtPi);
      q.rcp_sigma = 1.0 / problems[i].sigma_pp;
      q.rcp_modes = 1.0 / (double)m.n_modes;
      q.rcp_L = 1.0 / (double)m.L;
    }
    e = upload(&c->ppm, pm.data(), pm.size());
  }
  if (e == hipSuccess && n_inst > 1) {
    std::vector<int32_t> ri((size_t)c->ny);
    for (int i = 0; i < n_inst; ++i)
      for (int64_t j = 0; j < (int64_t)c->info[i].n_el + c->info[i].n_ph; ++j) ri[c->info[i].off + j] = i;
    e = upload(&c->row_inst, ri.data(), ri.size());
  }
  // integrator state and work vectors
  int64_t maxrows = 1;
  for (auto& in : c->info) maxrows = std::max<int64_t>(maxrows, (int64_t)in.n_el + in.n_ph);
  c->nchunk = (int)std::min<int64_t>(64, std::max<int64_t>(1, maxrows / 8192));
  const size_t ny = (size_t)std::max<int64_t>(c->ny, 1);
  for (int j = 0; j < 5 && e == hipSuccess; ++j) c->kbuf[j] = dalloc<double>(ny, &e);
  for (int j = 0; j < 2 && e == hipSuccess; ++j) c->zb[j] = dalloc<double>(ny, &e);
  for (int j = 0; j < 3 && e == hipSuccess; ++j) c->fs[j] = dalloc<double>(ny, &e);
  if (e == hipSuccess) c->ynew = dalloc<double>(ny, &e);
  if (e == hipSuccess) c->lte = dalloc<double>(ny, &e);
  if (e == hipSuccess) c->tmp = dalloc<double>(ny, &e);
  if (e == hipSuccess) c->tmp2 = dalloc<double>(ny, &e);
  if (e == hipSuccess) c->forcing = dalloc<double>(ny, &e);
  if (e == hipSuccess) c->partial = dalloc<double>(3 * (size_t)n_inst * c->nchunk, &e);
  if (e == hipSuccess) c->tvec = dalloc<double>(2 * (size_t)n_inst, &e);
  if (e == hipSuccess) c->summary_d = dalloc<int32_t>(2, &e);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->summary_h, 2 * sizeof(int32_t), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->scal_h, 8 * sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemset(c->forcing, 0, ny * sizeof(double));
  if (e == hipSuccess) c->st = dalloc<InstState>((size_t)n_inst, &e);
  if (e == hipSuccess) c->st_fast = dalloc<InstState>((size_t)n_inst, &e);
  if (e == hipSuccess) c->st_slow = dalloc<InstState>(1, &e);
  if (e == hipSuccess) c->health = dalloc<int32_t>((size_t)std::max(n_inst, 1), &e);
  if (e != hipSuccess) {
    fail(c, e == hipErrorOutOfMemory ? RTBTE_E_NOMEM : RTBTE_E_HIP, "work buffers: %s", hipGetErrorString(e));
    return cleanup(e == hipErrorOutOfMemory ? RTBTE_E_NOMEM : RTBTE_E_HIP);
  }
  c->group_rows_el = GE;
  c->group_rows_ph = GP;
  c->slots = std::max(GE, GP) == 1 ? 1 : (std::max(GE, GP) <= 8 ? 8 : 16);
  *out = c;
  if (rtbte_reset(c) != RTBTE_OK) {
    std::string msg = c->err;
    free_ctx(c);
    *out = nullptr;
    return fail(nullptr, RTBTE_E_HIP, "%s", msg.c_str());
  }
  return RTBTE_OK;
}

extern "C" void rtbte_destroy(rtbte_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  free_ctx(ctx);
}

extern "C" int rtbte_reset(rtbte_ctx* c) {
  if (!c) return RTBTE_E_INVAL;
  HIPCHK(c, hipSetDevice(c->device));
  std::vector<InstState> s((size_t)c->n_inst);
  for (auto& x : s) {
    std::memset(&x, 0, sizeof x);
    x.e1 = x.e2 = 1.0;
    x.first = 1;
    x.h_min = INFINITY;
    x.h_max = 0.0;
    x.done = 1;
  }
  HIPCHK(c, hipMemcpy(c->st, s.data(), s.size() * sizeof(InstState), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->st_fast, s.data(), s.size() * sizeof(InstState), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->st_slow, s.data(), sizeof(InstState), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemset(c->health, 0, (size_t)c->n_inst * sizeof(int32_t)));
  c->extra_rhs[0] = c->extra_rhs[1] = c->extra_rhs[2] = 0;
  c->slow_steps = 0;
  c->split_slow_evals = 0;
  c->last_status = 0;
  c->err64.assign((size_t)c->n_inst, -1.0);
  c->polls = 0;
  return RTBTE_OK;
}

extern "C" int rtbte_layout(const rtbte_ctx* c, int32_t inst, int64_t* y_offset, int32_t* n_el,
                            int32_t* n_ph) {
  if (!c || inst < 0 || inst >= c->n_inst) return RTBTE_E_INVAL;
  if (y_offset) *y_offset = c->info[inst].off;
  if (n_el) *n_el = c->info[inst].n_el;
  if (n_ph) *n_ph = c->info[inst].n_ph;
  return RTBTE_OK;
}

extern "C" int64_t rtbte_ny(const rtbte_ctx* c) { return c ? c->ny : -1; }

extern "C" int rtbte_counts(const rtbte_ctx* c, int32_t inst, int64_t counts[3]) {
  if (!c || !counts || inst < -1 || inst >= c->n_inst) return RTBTE_E_INVAL;
  counts[0] = counts[1] = counts[2] = 0;
  for (int i = 0; i < c->n_inst; ++i)
    if (inst < 0 || inst == i) {
      for (int k = 0; k < 3; ++k) counts[k] += c->counts[3 * i + k];
      counts[2] += c->folded[(size_t)i];
    }
  return RTBTE_OK;
}

extern "C" int rtbte_stored_counts(const rtbte_ctx* c, int32_t inst, int64_t counts[3]) {
  if (!c || !counts || inst < -1 || inst >= c->n_inst) return RTBTE_E_INVAL;
  counts[0] = counts[1] = counts[2] = 0;
  for (int i = 0; i < c->n_inst; ++i)
    if (inst < 0 || inst == i)
      for (int k = 0; k < 3; ++k) counts[k] += c->counts[3 * i + k];
  return RTBTE_OK;
}

extern "C" int rtbte_get_tuning(const rtbte_ctx* c, int32_t* group_rows_el, int32_t* group_rows_ph,
                                int64_t* item_channels) {
  if (!c) return RTBTE_E_INVAL;
  if (group_rows_el) *group_rows_el = c->group_rows_el;
  if (group_rows_ph) *group_rows_ph = c->group_rows_ph;
  if (item_channels) *item_channels = c->item_channels;
  return RTBTE_OK;
}

extern "C" int rtbte_get_tuning_source(const rtbte_ctx* c, int32_t* source, double* rhs_ms) {
  if (!c) return RTBTE_E_INVAL;
  if (source) *source = c->tuned;
  if (rhs_ms) *rhs_ms = c->tuned_ms;
  return RTBTE_OK;
}

extern "C" int64_t rtbte_graph_launches(const rtbte_ctx* c) { return c ? c->graph_launches : -1; }

extern "C" int rtbte_get_weight_format(const rtbte_ctx* c, int32_t* format, int32_t* bytes_per_channel,
                                       double* weight_rounding) {
  if (!c) return RTBTE_E_INVAL;
  int32_t f = c->wfmt, b = c->wfmt == -2 ? 12 : 16;
  double u = c->wfmt == -2 && c->f64_m < 52 ? std::ldexp(1.0, -(c->f64_m + 1)) : 0.0;
  if (c->mixed) {
    b = f == RTBTE_W_PACK8 ? 8 : 10;
    u = f == RTBTE_W_PACK8 ? std::ldexp(1.0, -(c->pack_m + 1))
        : f == RTBTE_W_F16X ? std::ldexp(1.0, -22)
        : f == RTBTE_W_F16  ? std::ldexp(1.0, -11)
                            : std::ldexp(1.0, -8);
  }
  if (format) *format = f;
  if (bytes_per_channel) *bytes_per_channel = b;
  if (weight_rounding) *weight_rounding = u;
  return RTBTE_OK;
}

// ------------------------------------------------------------ right-hand side
namespace {

// Algorithmic bytes of one collision-kernel launch: every stored channel of
// the selected parts once (FP64: 16 B plain, 12 B packed; mixed: 8 or 10 B
// and a 4 B scale per 512), the populations once (8 B per state; mixed: 4 B),
// the group and item tables, and the item row sums written.
double launch_bytes(const rtbte_ctx* c, int parts) {
  int64_t ch = 0, pp = 0;
  for (int i = 0; i < c->n_inst; ++i)
    for (int k = 0; k < 3; ++k)
      if (parts & (1 << k)) ch += c->counts[3 * i + k];
  if (c->ppm && (parts & 4)) {
    // matrix-free ph-ph channels stream their 8-byte words only
    for (int i = 0; i < c->n_inst; ++i) pp += c->counts[3 * i + 2];
    ch -= pp;
  }
  const double tables = (double)sizeof(Group) * (double)c->n_groups +
                        (double)(sizeof(Item) + 4 + 8 * kMaxGroupRows) * (double)c->n_items;
  if (c->mixed)
    return (c->wfmt == RTBTE_W_PACK8 ? 8.0 : 10.0) * (double)ch + 4.0 * (double)ch / kMixBlock +
           8.0 * (double)pp + 4.0 * (double)c->ny + tables;
  return (c->pk ? 12.0 : 16.0) * (double)ch + 8.0 * (double)pp + 8.0 * (double)c->ny + tables;
}

hipError_t harvest(rtbte_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0.f;
    hipError_t e = hipEventElapsedTime(&ms, p.a, p.b);
    if (e != hipSuccess) return e;
    c->prof_ms += ms;
    c->prof_bytes += p.bytes;
    c->prof_n++;
    c->pool.emplace_back(p.a, p.b);
  }
  c->pending.clear();
  return hipSuccess;
}

// The right-hand side in two launches: per-item row sums (the collision
// kernel, the one that streams the channels and is timed when profiling),
// then the per-row sums of items with the plain or stage epilogue.
// fp64: use the FP64 lists of a mixed context that keeps them (not timed).
// partial, popf: scratch to use instead of the context's own (the
// allocation-free entry point; its launches are never timed).
hipError_t rhs_launch(rtbte_ctx* c, const double* z, int parts, const InstState* st, const FinishArgs& f,
                      bool stage, hipStream_t s, bool deriv = false, bool fp64 = false,
                      double* partial = nullptr, float* popf = nullptr) {
  const bool use_mixed = c->mixed && !fp64;
  const bool own = partial == nullptr;
  if (own) {
    partial = c->partial_items;
    popf = c->popf;
  }
  RowArgs a{};
  a.deriv = deriv ? 1 : 0;
  a.ch = c->ch;
  a.pk = c->pk;
  a.pkw = c->pkw;
  a.pack_p = c->pack_p;
  a.pack_m = c->f64_m;
  a.info = c->info_d;
  a.groups = c->groups;
  a.items = c->items;
  a.order = c->order;
  a.n_items = c->n_items;
  a.parts = parts;
  a.z = z;
  a.partial = partial;
  a.st = st;
  a.ny = c->ny;
  a.ppm = c->ppm;
  a.hw = c->energy_d;
  if (c->tiled && !c->mixed) {
    a.blocks = c->tblocks;
    a.border = c->border;
    a.n_blocks = c->n_blocks;
    a.tiles = c->tiles;
    a.bnd = c->bnd;
  }
  MixArgs m{};
  if (use_mixed) {
    m.idx = c->mix_idx;
    m.wq = c->mix_wq;
    m.scale = c->mix_scale;
    m.n_scale = (c->n_ch + kMixBlock - 1) / kMixBlock;
    m.pop = popf;
    m.groups = c->groups;
    m.items = c->items;
    m.order = c->order;
    m.n_items = c->n_items;
    m.parts = parts;
    m.wfmt = c->wfmt;
    m.pack_p = c->pack_p;
    m.pack_m = c->pack_m;
    m.info = c->info_d;
    m.partial = partial;
    m.st = st;
    m.ny = c->ny;
    m.ppm = c->ppm;
    m.hw = c->energy_d;
    if (c->tiled) {
      m.blocks = c->tblocks;
      m.border = c->border;
      m.n_blocks = c->n_blocks;
      m.tiles = c->tiles;
      m.bnd = c->bnd;
    }
  }
  auto launch = [&]() {
    if (!use_mixed) return launch_items(a, c->slots, s);
    hipError_t e2 = launch_popf(popf, z, c->row_group, c->groups, c->ny, s);
    return e2 == hipSuccess ? launch_items_mixed(m, c->slots, s) : e2;
  };
  hipError_t e;
  if (!c->prof || fp64 || !own) {
    e = launch();
  } else {
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (!c->pool.empty()) {
      ev = c->pool.back();
      c->pool.pop_back();
    } else {
      e = hipEventCreate(&ev.first);
      if (e == hipSuccess) e = hipEventCreate(&ev.second);
      if (e != hipSuccess) return e;
    }
    e = hipEventRecord(ev.first, s);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(ev.second, s);
    c->pending.push_back({ev.first, ev.second, launch_bytes(c, parts)});
  }
  if (e != hipSuccess) return e;
  FinishArgs fa = f;
  fa.groups = c->groups;
  fa.row_group = c->row_group;
  fa.item_ptr = c->item_ptr;
  fa.partial = partial;
  fa.n_rows = c->ny;
  return launch_finish_rows(fa, stage, s);
}

}  // namespace

namespace {

// Mixed-precision right-hand side against the FP64 lists kept beside it, at
// the state y: err64[inst] = ||f_mixed - f_fp64|| / ||f_fp64|| (2-norms over
// the instance's rows).  Diagnostic launches: not counted, not timed.
int check_fp64(rtbte_ctx* c, const double* y, hipStream_t s) {
  FinishArgs f{};
  f.out = c->tmp;
  HIPCHK(c, rhs_launch(c, y, RTBTE_PART_ALL, nullptr, f, false, s));
  f.out = c->tmp2;
  HIPCHK(c, rhs_launch(c, y, RTBTE_PART_ALL, nullptr, f, false, s, false, true));
  HIPCHK(c, launch_diff_norms(c->tmp, c->tmp2, c->info_d, c->partial, c->n_inst, c->nchunk, s));
  std::vector<double> part(2 * (size_t)c->n_inst * c->nchunk);
  HIPCHK(c, hipMemcpyAsync(part.data(), c->partial, part.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  for (int i = 0; i < c->n_inst; ++i) {
    double d2 = 0.0, b2 = 0.0;
    for (int j = 0; j < c->nchunk; ++j) {
      d2 += part[2 * ((size_t)i * c->nchunk + j)];
      b2 += part[2 * ((size_t)i * c->nchunk + j) + 1];
    }
    c->err64[(size_t)i] = b2 > 0.0 ? std::sqrt(d2 / b2) : (d2 > 0.0 ? INFINITY : 0.0);
  }
  return RTBTE_OK;
}

}  // namespace

extern "C" int rtbte_check_fp64(rtbte_ctx* c, const double* y, double* err, void* stream) {
  TraceRange tr("rtbte_check_fp64");
  if (!c) return RTBTE_E_INVAL;
  if (!c->mixed || !c->keep64)
    return fail(c, RTBTE_E_UNSUPPORTED, "rtbte_check_fp64 needs an RTBTE_MIXED context created with fp64_check > 0");
  if (!y) return fail(c, RTBTE_E_INVAL, "rtbte_check_fp64: bad arguments");
  HIPCHK(c, hipSetDevice(c->device));
  int rc = check_fp64(c, y, (hipStream_t)stream);
  if (rc == RTBTE_OK && err)
    for (int i = 0; i < c->n_inst; ++i) err[i] = c->err64[(size_t)i];
  return rc;
}

extern "C" int rtbte_rates(rtbte_ctx* c, const double* y, double* rates, int32_t parts, void* stream) {
  TraceRange tr("rtbte_rates");
  if (!c) return RTBTE_E_INVAL;
  if (c->mixed) return fail(c, RTBTE_E_UNSUPPORTED, "rtbte_rates needs an RTBTE_FP64 context");
  if (!y || !rates || parts < 1 || parts > 7) return fail(c, RTBTE_E_INVAL, "rtbte_rates: bad arguments");
  if (y == rates) return fail(c, RTBTE_E_INVAL, "rtbte_rates: y and rates must not overlap");
  HIPCHK(c, hipSetDevice(c->device));
  FinishArgs f{};
  f.out = rates;
  HIPCHK(c, rhs_launch(c, y, parts, nullptr, f, false, (hipStream_t)stream, true));
  return RTBTE_OK;
}

extern "C" int rtbte_rhs(rtbte_ctx* c, const double* y, double* ydot, int32_t parts, void* stream) {
  TraceRange tr("rtbte_rhs");
  if (!c) return RTBTE_E_INVAL;
  if (!y || !ydot || parts < 1 || parts > 7) return fail(c, RTBTE_E_INVAL, "rtbte_rhs: bad arguments");
  if (y == ydot) return fail(c, RTBTE_E_INVAL, "rtbte_rhs: y and ydot must not overlap");
  HIPCHK(c, hipSetDevice(c->device));
  FinishArgs f{};
  f.out = ydot;
  HIPCHK(c, rhs_launch(c, y, parts, nullptr, f, false, (hipStream_t)stream));
  for (int k = 0; k < 3; ++k)
    if (parts & (1 << k)) c->extra_rhs[k]++;
  return RTBTE_OK;
}

// rtbte_rhs with its scratch in the static device buffer: the same kernels,
// no allocation of any kind.  Nothing in the scratch has to start at zero:
// every item row sum and population code a call reads is written earlier in
// the same call.
extern "C" int rtbte_rhs_noalloc(rtbte_ctx* c, const double* y, double* ydot, int32_t parts, void* stream) {
  if (!c) return RTBTE_E_INVAL;
  if (!y || !ydot || parts < 1 || parts > 7) return fail(c, RTBTE_E_INVAL, "rtbte_rhs_noalloc: bad arguments");
  if (y == ydot) return fail(c, RTBTE_E_INVAL, "rtbte_rhs_noalloc: y and ydot must not overlap");
  const size_t need = noalloc_scratch_bytes(c->n_items, c->ny, c->mixed);
  if (need > kStaticScratchBytes)
    return fail(c, RTBTE_E_INVAL,
                "rtbte_rhs_noalloc: this context needs %zu bytes of scratch, more than the static %zu "
                "(%lld work items, %lld states); use rtbte_rhs", need, kStaticScratchBytes,
                (long long)c->n_items, (long long)c->ny);
  if (!c->scratch_dev) return fail(c, RTBTE_E_HIP, "rtbte_rhs_noalloc: static scratch not set up");
  HIPCHK(c, hipSetDevice(c->device));
  unsigned char* base = static_cast<unsigned char*>(c->scratch_dev);
  double* sums = reinterpret_cast<double*>(base);
  float* codes = c->mixed ? reinterpret_cast<float*>(base + noalloc_scratch_bytes(c->n_items, c->ny, false))
                          : nullptr;
  FinishArgs f{};
  f.out = ydot;
  HIPCHK(c, rhs_launch(c, y, parts, nullptr, f, false, (hipStream_t)stream, false, false, sums, codes));
  for (int k = 0; k < 3; ++k)
    if (parts & (1 << k)) c->extra_rhs[k]++;
  return RTBTE_OK;
}

extern "C" int64_t rtbte_noalloc_scratch_bytes(const rtbte_ctx* c) {
  if (!c) return -1;
  return (int64_t)noalloc_scratch_bytes(c->n_items, c->ny, c->mixed);
}

extern "C" int64_t rtbte_noalloc_scratch_limit(void) { return (int64_t)kStaticScratchBytes; }

// ---------------------------------------------------------------- integrators
namespace {

Ctl make_ctl(const rtbte_options& o, bool fast, bool fixed) {
  Ctl t{};
  t.k1 = o.pid_k1;
  t.k2 = o.pid_k2;
  t.k3 = o.pid_k3;
  t.order = o.pid_order;
  t.safety = o.safety;
  t.eta_max = o.eta_max;
  t.eta_max_first = o.eta_max_first;
  t.eta_fail_min = o.eta_fail_min;
  t.eta_fail_max = o.eta_fail_max;
  t.eta_fail_repeat = o.eta_fail_repeat;
  t.small_nef = o.small_nef;
  t.eps_floor = o.eps_floor;
  t.rtol = fast ? o.fast_rtol : o.rtol;
  t.atol_el = fast ? o.fast_atol_el : o.atol_el;
  t.atol_ph = fast ? o.fast_atol_ph : o.atol_ph;
  t.max_fails = o.max_fails;
  t.alt_sign = o.pid_alt_sign;
  t.fixed = fixed ? 1 : 0;
  t.stages = fixed ? 4 : 5;
  return t;
}

// Enqueue one attempted step of tableau `tb` for every live instance of `st`.
int enqueue_step(rtbte_ctx* c, double* y, int parts, const double* forcing, InstState* st,
                 const Ctl& ctl, const Tableau& tb, hipStream_t s) {
  FinishArgs f{};
  f.y = y;
  f.st = st;
  f.forcing = forcing;
  for (int j = 0; j < 5; ++j) f.k[j] = c->kbuf[j];
  for (int i = 0; i < tb.S; ++i) {
    const double* z = i == 0 ? y : c->zb[i % 2];
    f.zout = c->zb[(i + 1) % 2];
    f.stage = i;
    f.last = i == tb.S - 1;
    for (int j = 0; j < 5; ++j) {
      f.a[j] = (!f.last && j <= i) ? tb.A[i + 1][j] : 0.0;
      f.b[j] = tb.b[j];
      f.d[j] = tb.d[j];
    }
    f.ynew = c->ynew;
    f.lte = c->lte;
    HIPCHK(c, rhs_launch(c, z, parts, st, f, true, s));
  }
  if (tb.embedded) {
    HIPCHK(c, launch_wrms(c->lte, y, c->info_d, st, c->partial, c->n_inst, c->nchunk, ctl, s));
  } else {
    // fixed steps: the RMS of the candidate state, so that a step that
    // diverges (a non-finite or overflowing state) is caught and not committed
    Ctl rms = ctl;
    rms.rtol = 0.0;
    rms.atol_el = rms.atol_ph = 1.0;
    HIPCHK(c, launch_wrms(c->ynew, y, c->info_d, st, c->partial, c->n_inst, c->nchunk, rms, s));
  }
  HIPCHK(c, launch_control(st, c->partial, c->info_d, c->n_inst, c->nchunk, ctl, s));
  HIPCHK(c, launch_commit(y, c->ynew, c->row_inst, st, c->ny, s));
  return RTBTE_OK;
}

// Starting step (Hairer-Norsett-Wanner) for instances flagged need_h0.
int enqueue_h0(rtbte_ctx* c, double* y, int parts, const double* forcing, InstState* st, const Ctl& ctl,
               hipStream_t s) {
  const size_t np = (size_t)c->n_inst * c->nchunk;
  double* py = c->partial;
  double* pf = c->partial + np;
  FinishArgs f{};
  f.out = c->tmp;  // f0
  HIPCHK(c, rhs_launch(c, y, parts, nullptr, f, false, s));
  if (forcing) {
    const double* v[2] = {c->tmp, forcing};
    const double cf[2] = {1.0, 1.0};
    for (int i = 0; i < c->n_inst; ++i)
      HIPCHK(c, launch_lincomb(c->tmp, v, cf, 2, c->info[i].off + c->info[i].n_el, c->info[i].n_ph, s));
  }
  HIPCHK(c, launch_wrms(y, y, c->info_d, nullptr, py, c->n_inst, c->nchunk, ctl, s));
  HIPCHK(c, launch_wrms(c->tmp, y, c->info_d, nullptr, pf, c->n_inst, c->nchunk, ctl, s));
  HIPCHK(c, launch_h0_stage1(st, py, pf, c->info_d, c->n_inst, c->nchunk, s));
  HIPCHK(c, launch_h0_axpy(c->zb[0], y, c->tmp, c->row_inst, st, c->ny, s));
  f.out = c->tmp2;  // f1
  HIPCHK(c, rhs_launch(c, c->zb[0], parts, nullptr, f, false, s));
  if (forcing) {
    const double* v[2] = {c->tmp2, forcing};
    const double cf[2] = {1.0, 1.0};
    for (int i = 0; i < c->n_inst; ++i)
      HIPCHK(c, launch_lincomb(c->tmp2, v, cf, 2, c->info[i].off + c->info[i].n_el, c->info[i].n_ph, s));
  }
  HIPCHK(c, launch_sub(c->tmp2, c->tmp2, c->tmp, c->ny, s));
  HIPCHK(c, launch_wrms(c->tmp2, y, c->info_d, nullptr, py, c->n_inst, c->nchunk, ctl, s));
  HIPCHK(c, launch_h0_stage2(st, py, c->info_d, c->n_inst, c->nchunk, (double)c->opt.pid_order, s));
  for (int k = 0; k < 3; ++k)
    if (parts & (1 << k)) c->extra_rhs[k] += 2;
  return RTBTE_OK;
}

bool same_ctl(const Ctl& a, const Ctl& b) {
  return a.k1 == b.k1 && a.k2 == b.k2 && a.k3 == b.k3 && a.order == b.order && a.safety == b.safety &&
         a.eta_max == b.eta_max && a.eta_max_first == b.eta_max_first && a.eta_fail_min == b.eta_fail_min &&
         a.eta_fail_max == b.eta_fail_max && a.eps_floor == b.eps_floor && a.rtol == b.rtol &&
         a.eta_fail_repeat == b.eta_fail_repeat && a.small_nef == b.small_nef &&
         a.atol_el == b.atol_el && a.atol_ph == b.atol_ph && a.max_fails == b.max_fails &&
         a.alt_sign == b.alt_sign && a.fixed == b.fixed && a.stages == b.stages;
}

// The executable graph of `steps` attempted steps with these arguments,
// captured on the context's own stream the first time it is asked for.  The
// captured region holds kernel launches only.
int step_graph(rtbte_ctx* c, double* y, int parts, const double* forcing, InstState* st, const Ctl& ctl,
               const Tableau& tb, int steps, hipGraphExec_t* out) {
  for (auto& g : c->graphs) {
    const auto& k = g.key;
    if (k.y == y && k.forcing == forcing && k.st == st && k.tb_stages == tb.S && k.parts == parts &&
        k.steps == steps && same_ctl(k.ctl, ctl)) {
      *out = g.exec;
      return RTBTE_OK;
    }
  }
  if (!c->cap) HIPCHK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  if (c->graphs.size() >= 16) {
    (void)hipGraphExecDestroy(c->graphs.front().exec);
    (void)hipGraphDestroy(c->graphs.front().g);
    c->graphs.erase(c->graphs.begin());
  }
  HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  int rc = RTBTE_OK;
  for (int m = 0; m < steps && rc == RTBTE_OK; ++m) rc = enqueue_step(c, y, parts, forcing, st, ctl, tb, c->cap);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->cap, &g);
  if (rc != RTBTE_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return rc != RTBTE_OK ? rc : fail(c, RTBTE_E_HIP, "step capture: %s", hipGetErrorString(e));
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e2 != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(c, RTBTE_E_HIP, "graph instantiate: %s", hipGetErrorString(e2));
  }
  rtbte_ctx::GraphEntry ent{};
  ent.key = {y, forcing, st, tb.S, parts, steps, ctl};
  ent.g = g;
  ent.exec = ex;
  c->graphs.push_back(ent);
  *out = ex;
  return RTBTE_OK;
}

int poll(rtbte_ctx* c, InstState* st, int n_st, double* t, double* h, hipStream_t s, bool* all_done, int* worst) {
  HIPCHK(c, launch_finish(st, t, h, n_st, c->summary_d, s));
  HIPCHK(c, hipMemcpyAsync(c->summary_h, c->summary_d, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (c->prof) HIPCHK(c, harvest(c));
  *all_done = c->summary_h[0] != 0;
  *worst = c->summary_h[1];
  return RTBTE_OK;
}

// Run an integrator on `st` until every instance is done.
int run(rtbte_ctx* c, double* y, double* t, double* h, double t_out, int one_step, int parts,
        const double* forcing, InstState* st, const Ctl& ctl, const Tableau& tb, double h_cap,
        int64_t fixed_steps, double fixed_h, hipStream_t s) {
  HIPCHK(c, launch_begin(st, t, h, c->n_inst, t_out, one_step, h_cap, fixed_steps, fixed_h, s));
  if (h && fixed_steps <= 0) {
    // the starting-step estimate (two right-hand sides) only when an
    // instance that still has to move asks for it
    std::vector<double> hh((size_t)c->n_inst), tt((size_t)c->n_inst);
    HIPCHK(c, hipMemcpyAsync(hh.data(), h, hh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(tt.data(), t, tt.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    bool need = false;
    for (size_t i = 0; i < hh.size(); ++i) need |= !(hh[i] > 0.0) && tt[i] < t_out;
    if (need) {
      int rc = enqueue_h0(c, y, parts, forcing, st, ctl, s);
      if (rc) return rc;
    }
  }
  const int per_poll = one_step ? 1 : c->opt.steps_per_poll;
  bool done = false;
  int worst = 0;
  // Graph replay: the same launches as the loop below, captured once per
  // argument set (profiling times individual launches, so it stays eager).
  const bool graph = c->opt.use_graph && !c->prof;
  // a fixed-step run launches exactly its steps (no attempts that find
  // every instance done at the end of the last poll interval)
  int64_t left = fixed_steps;
  while (!done) {
    TraceRange tr_poll("rtbte poll interval");
    const int n = fixed_steps > 0 && left > 0 ? (int)std::min<int64_t>(per_poll, left) : per_poll;
    if (fixed_steps > 0) left -= n;
    if (graph) {
      hipGraphExec_t ex = nullptr;
      int rc = step_graph(c, y, parts, forcing, st, ctl, tb, n, &ex);
      if (rc) return rc;
      HIPCHK(c, hipGraphLaunch(ex, s));
      c->graph_launches++;
    } else {
      for (int m = 0; m < n; ++m) {
        int rc = enqueue_step(c, y, parts, forcing, st, ctl, tb, s);
        if (rc) return rc;
      }
    }
    HIPCHK(c, launch_health(y, c->info_d, c->health, c->n_inst, kHealthTol, s));
    int rc = poll(c, st, c->n_inst, t, h, s, &done, &worst);
    if (rc) return rc;
    if (c->keep64 && ++c->polls >= c->opt.fp64_check) {
      c->polls = 0;
      rc = check_fp64(c, y, s);
      if (rc) return rc;
    }
  }
  c->last_status = worst;
  if (worst == RTBTE_E_STEP) return fail(c, RTBTE_E_STEP, "too many consecutive error-test failures");
  if (worst == RTBTE_E_NONFINITE) return fail(c, RTBTE_E_NONFINITE, "non-finite error estimate");
  return RTBTE_OK;
}

}  // namespace

extern "C" int rtbte_step_adaptive(rtbte_ctx* c, double* y, double* t, double* h, double t_out,
                                   int32_t one_step, void* stream) {
  TraceRange tr("rtbte_step_adaptive");
  if (!c) return RTBTE_E_INVAL;
  if (!y || !t || !h || !std::isfinite(t_out)) return fail(c, RTBTE_E_INVAL, "step_adaptive: bad arguments");
  HIPCHK(c, hipSetDevice(c->device));
  const Ctl ctl = make_ctl(c->opt, false, false);
  return run(c, y, t, h, t_out, one_step ? 1 : 0, RTBTE_PART_ALL, nullptr, c->st, ctl, zonneveld(), 0.0,
             0, 0.0, (hipStream_t)stream);
}

extern "C" int rtbte_step_rk4(rtbte_ctx* c, double* y, double* t, double h_step, int64_t n_steps,
                              void* stream) {
  TraceRange tr("rtbte_step_rk4");
  if (!c) return RTBTE_E_INVAL;
  if (!y || !t || !(h_step > 0) || n_steps < 0) return fail(c, RTBTE_E_INVAL, "step_rk4: bad arguments");
  if (n_steps == 0) return RTBTE_OK;
  HIPCHK(c, hipSetDevice(c->device));
  const Ctl ctl = make_ctl(c->opt, false, true);
  return run(c, y, t, nullptr, 0.0, 0, RTBTE_PART_ALL, nullptr, c->st, ctl, rk4(), 0.0, n_steps, h_step,
             (hipStream_t)stream);
}

namespace {

// Fixed RK4 substeps of h over [t0, t1] on `parts` (plus `forcing` on the
// phonon rows, if given), the last substep cut to land on t1; runs on the
// fast-integrator state with the device clocks t_in (one per instance).
int rk4_segment(rtbte_ctx* c, double* y, double* t_in, int parts, const double* forcing, const Ctl& ctl,
                double t0, double t1, double h, hipStream_t s) {
  const Tableau tb = rk4();
  int64_t nfull = 0;
  double tt = t0;
  while (tt < t1) {
    if (tt + h >= t1) break;
    tt += h;
    ++nfull;
  }
  HIPCHK(c, launch_fill(t_in, t0, c->n_inst, s));
  int rc = RTBTE_OK;
  if (nfull > 0) rc = run(c, y, t_in, nullptr, 0.0, 0, parts, forcing, c->st_fast, ctl, tb, 0.0, nfull, h, s);
  if (rc == RTBTE_OK && t1 - tt > 0) {
    HIPCHK(c, launch_fill(t_in, tt, c->n_inst, s));
    rc = run(c, y, t_in, nullptr, 0.0, 0, parts, forcing, c->st_fast, ctl, tb, 0.0, 1, t1 - tt, s);
  }
  return rc;
}

}  // namespace

namespace {

// One MIS slow step of size hs from tc (Methods, MRI method): slow
// right-hand sides at the stage values, each stage interval integrated by the
// fast solver (adaptive ERK on st_fast with the device step h_in carried
// along, or fixed RK4 substeps) with the constant forcing of Eq. (mis_coef).
int mis_one(rtbte_ctx* c, double* y, double tc, double hs, bool fixed, const Ctl& ctl, const Tableau& tb,
            hipStream_t s) {
  double* t_in = c->tvec;               // fast solver clocks (one per instance)
  double* h_in = c->tvec + c->n_inst;   // fast solver steps (one per instance)
  FinishArgs f{};
  f.out = c->fs[0];
  HIPCHK(c, rhs_launch(c, y, RTBTE_PART_PHPH, nullptr, f, false, s));
  c->extra_rhs[2]++;
  for (int i = 1; i < 4; ++i) {
    const double* v[3] = {c->fs[0], c->fs[1], c->fs[2]};
    for (int k = 0; k < c->n_inst; ++k)
      HIPCHK(c, launch_lincomb(c->forcing, v, MIS_R[i], i, c->info[k].off + c->info[k].n_el, c->info[k].n_ph, s));
    const double t0 = tc + MIS_C[i - 1] * hs, t1 = tc + MIS_C[i] * hs;
    if (!fixed) HIPCHK(c, launch_fill(t_in, t0, c->n_inst, s));
    int rc;
    if (!fixed) {
      rc = run(c, y, t_in, h_in, t1, 0, RTBTE_PART_EPH | RTBTE_PART_PHE, c->forcing, c->st_fast, ctl, tb,
               t1 - t0, 0, 0.0, s);
    } else {
      rc = rk4_segment(c, y, t_in, RTBTE_PART_EPH | RTBTE_PART_PHE, c->forcing, ctl, t0, t1, c->opt.h_fast, s);
    }
    if (rc) return rc;
    if (i < 3) {
      f.out = c->fs[i];
      HIPCHK(c, rhs_launch(c, y, RTBTE_PART_PHPH, nullptr, f, false, s));
      c->extra_rhs[2]++;
    }
  }
  return RTBTE_OK;
}

// Checks shared by the multirate entry points; reads t to the host (every
// instance must be at the same time: the slow steps are common) and h_fast
// into the fast solvers' step slots.
int mis_setup(rtbte_ctx* c, double* y, double* t, double* h_fast, double t_out, const char* who, bool* fixed,
              Ctl* ctl, Tableau* tb, double* tc, hipStream_t s) {
  if (!y || !t || !h_fast || !std::isfinite(t_out)) return fail(c, RTBTE_E_INVAL, "%s: bad arguments", who);
  HIPCHK(c, hipSetDevice(c->device));
  *fixed = c->opt.fast_mode == 1;
  if (*fixed && !(c->opt.h_fast > 0)) return fail(c, RTBTE_E_INVAL, "fixed fast mode needs h_fast > 0");
  *ctl = make_ctl(c->opt, true, *fixed);
  *tb = *fixed ? rk4() : zonneveld();
  std::vector<double> th((size_t)c->n_inst);
  HIPCHK(c, hipMemcpyAsync(th.data(), t, th.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(c->tvec + c->n_inst, h_fast, (size_t)c->n_inst * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipStreamSynchronize(s));
  for (double v : th)
    if (v != th[0]) return fail(c, RTBTE_E_UNSUPPORTED, "%s: every instance must start at the same time", who);
  *tc = th[0];
  return RTBTE_OK;
}

}  // namespace

extern "C" int rtbte_step_multirate(rtbte_ctx* c, double* y, double* t, double* h_fast, double t_out,
                                    double h_slow, int32_t one_step, void* stream) {
  TraceRange tr("rtbte_step_multirate");
  if (!c) return RTBTE_E_INVAL;
  if (!(h_slow > 0)) return fail(c, RTBTE_E_INVAL, "step_multirate: bad arguments");
  hipStream_t s = (hipStream_t)stream;
  bool fixed = false;
  Ctl ctl{};
  Tableau tb{};
  double tc = 0.0;
  int rc = mis_setup(c, y, t, h_fast, t_out, "step_multirate", &fixed, &ctl, &tb, &tc, s);
  if (rc) return rc;
  if (!c->mis_keep) {
    hipError_t e = hipMalloc((void**)&c->mis_keep, (size_t)c->ny * sizeof(double));
    if (e != hipSuccess) {
      c->mis_keep = nullptr;
      return fail(c, RTBTE_E_NOMEM, "step_multirate: %s", hipGetErrorString(e));
    }
  }
  const size_t nb = (size_t)c->ny * sizeof(double);
  while (tc < t_out) {
    double hs = h_slow;
    const bool last = tc + hs >= t_out;
    if (last) hs = t_out - tc;
    // the fast solves advance y in place: keep the step's starting state so
    // that a failure leaves y and t at the start of the failing slow step
    HIPCHK(c, hipMemcpyAsync(c->mis_keep, y, nb, hipMemcpyDeviceToDevice, s));
    rc = mis_one(c, y, tc, hs, fixed, ctl, tb, s);
    if (rc) {
      (void)hipMemcpyAsync(y, c->mis_keep, nb, hipMemcpyDeviceToDevice, s);
      (void)launch_fill(t, tc, c->n_inst, s);
      (void)hipStreamSynchronize(s);
      return rc;
    }
    tc = last ? t_out : tc + hs;
    c->slow_steps++;
    if (one_step) break;
  }
  HIPCHK(c, launch_fill(t, tc, c->n_inst, s));
  if (!fixed)
    HIPCHK(c, hipMemcpyAsync(h_fast, c->tvec + c->n_inst, (size_t)c->n_inst * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return RTBTE_OK;
}

extern "C" int rtbte_step_multirate_adaptive(rtbte_ctx* c, double* y, double* t, double* h_fast, double* h_slow,
                                             double t_out, int32_t one_step, void* stream) {
  TraceRange tr("rtbte_step_multirate_adaptive");
  if (!c) return RTBTE_E_INVAL;
  if (!h_slow) return fail(c, RTBTE_E_INVAL, "step_multirate_adaptive: bad arguments");
  hipStream_t s = (hipStream_t)stream;
  bool fixed = false;
  Ctl ctl{};
  Tableau tb{};
  double tc = 0.0;
  int rc = mis_setup(c, y, t, h_fast, t_out, "step_multirate_adaptive", &fixed, &ctl, &tb, &tc, s);
  if (rc) return rc;
  const int n_inst = c->n_inst;
  std::vector<double> hs((size_t)n_inst);
  HIPCHK(c, hipMemcpyAsync(hs.data(), h_slow, hs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (!(hs[0] > 0.0) || !std::isfinite(hs[0]))
    return fail(c, RTBTE_E_INVAL, "step_multirate_adaptive: the slow step h_slow must be positive");
  for (double v : hs)
    if (v != hs[0])
      return fail(c, RTBTE_E_UNSUPPORTED, "step_multirate_adaptive: every instance must start with the same slow step");
  static_assert(sizeof(InstInfo) <= 2 * sizeof(double), "selected-instance slot");
  if (!c->mra) {
    hipError_t e = hipMalloc((void**)&c->mra, (3 * (size_t)c->ny + (size_t)c->nchunk + 2) * sizeof(double));
    if (e != hipSuccess) {
      c->mra = nullptr;
      return fail(c, RTBTE_E_NOMEM, "step_multirate_adaptive: %s", hipGetErrorString(e));
    }
  }
  double* y_full = c->mra;
  double* y_half = c->mra + c->ny;
  double* est = c->mra + 2 * c->ny;
  double* sel_partial = c->mra + 3 * c->ny;
  InstInfo* sel_info = reinterpret_cast<InstInfo*>(sel_partial + c->nchunk);
  // slow controller: I control on the step-doubling estimate of the
  // third-order MIS step, eta = safety eps^(-1/4), the options' tolerances;
  // one controller state for the whole context (the slow steps are common)
  Ctl cs = make_ctl(c->opt, false, false);
  cs.k1 = 1.0;
  cs.k2 = 0.0;
  cs.k3 = 0.0;
  cs.order = 4.0;
  cs.alt_sign = 0;
  cs.stages = 0;  // right-hand sides are counted by the MIS steps
  HIPCHK(c, launch_begin(c->st_slow, t, h_slow, 1, t_out, one_step ? 1 : 0, 0.0, 0, 0.0, s));
  const size_t nb = (size_t)c->ny * sizeof(double);
  for (;;) {
    InstState st{};
    HIPCHK(c, hipMemcpyAsync(&st, c->st_slow, sizeof st, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (st.done) break;
    const double H = st.h_use;
    tc = st.t;
    HIPCHK(c, hipMemcpyAsync(y_full, y, nb, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(y_half, y, nb, hipMemcpyDeviceToDevice, s));
    rc = mis_one(c, y_full, tc, H, fixed, ctl, tb, s);
    if (rc == RTBTE_OK) rc = mis_one(c, y_half, tc, 0.5 * H, fixed, ctl, tb, s);
    if (rc == RTBTE_OK) rc = mis_one(c, y_half, tc + 0.5 * H, 0.5 * H, fixed, ctl, tb, s);
    if (rc) break;   // y is still the last accepted state (the attempts ran on copies)
    // estimate (y_half - y_full) / (2^3 - 1); weights from the attempt's start
    const double* dv[2] = {y_half, y_full};
    const double one_m[2] = {1.0, -1.0}, seventh[1] = {1.0 / 7.0};
    const double* ev[1] = {est};
    HIPCHK(c, launch_lincomb(est, dv, one_m, 2, 0, c->ny, s));
    HIPCHK(c, launch_lincomb(est, ev, seventh, 1, 0, c->ny, s));
    if (n_inst == 1) {
      HIPCHK(c, launch_wrms(est, y, c->info_d, c->st_slow, c->partial, 1, c->nchunk, cs, s));
      HIPCHK(c, launch_control(c->st_slow, c->partial, c->info_d, 1, c->nchunk, cs, s));
    } else {
      // every instance's norm, then the controller on the largest
      HIPCHK(c, launch_wrms(est, y, c->info_d, nullptr, c->partial, n_inst, c->nchunk, cs, s));
      HIPCHK(c, launch_select_max_norm(c->partial, c->info_d, n_inst, c->nchunk, sel_partial, sel_info, s));
      HIPCHK(c, launch_control(c->st_slow, sel_partial, sel_info, 1, c->nchunk, cs, s));
    }
    HIPCHK(c, launch_commit(y, y_half, nullptr, c->st_slow, c->ny, s));
    bool done = false;
    int worst = 0;
    rc = poll(c, c->st_slow, 1, t, h_slow, s, &done, &worst);
    if (rc) return rc;
    if (done) {
      c->last_status = worst;
      if (worst == RTBTE_E_STEP) rc = fail(c, RTBTE_E_STEP, "too many consecutive slow-step failures");
      if (worst == RTBTE_E_NONFINITE) rc = fail(c, RTBTE_E_NONFINITE, "non-finite slow error estimate");
      break;
    }
  }
  // the common clock and slow step to every instance
  HIPCHK(c, launch_broadcast_first(t, n_inst, s));
  HIPCHK(c, launch_broadcast_first(h_slow, n_inst, s));
  if (!fixed)
    HIPCHK(c, hipMemcpyAsync(h_fast, c->tvec + n_inst, (size_t)n_inst * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return rc;
}

extern "C" int rtbte_step_split(rtbte_ctx* c, double* y, double* t, double h_fast, double h_slow, double t_out,
                                void* stream) {
  TraceRange tr("rtbte_step_split");
  if (!c) return RTBTE_E_INVAL;
  if (!y || !t || !(h_fast > 0) || !(h_slow > 0) || !std::isfinite(t_out))
    return fail(c, RTBTE_E_INVAL, "step_split: bad arguments");
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  const Ctl ctl = make_ctl(c->opt, true, true);
  std::vector<double> th((size_t)c->n_inst);
  HIPCHK(c, hipMemcpyAsync(th.data(), t, th.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  for (double v : th)
    if (v != th[0]) return fail(c, RTBTE_E_UNSUPPORTED, "step_split: every instance must start at the same time");
  double tc = th[0];
  double* t_in = c->tvec;
  while (tc < t_out) {
    double hs = h_slow;
    const bool last = tc + hs >= t_out;
    if (last) hs = t_out - tc;
    // fast part over the step, then the slow part over the same interval
    int rc = rk4_segment(c, y, t_in, RTBTE_PART_EPH | RTBTE_PART_PHE, nullptr, ctl, 0.0, hs, h_fast, s);
    if (rc == RTBTE_OK) rc = rk4_segment(c, y, t_in, RTBTE_PART_PHPH, nullptr, ctl, 0.0, hs, hs, s);
    if (rc) return rc;
    c->split_slow_evals += 4;
    tc = last ? t_out : tc + hs;
    c->slow_steps++;
  }
  HIPCHK(c, launch_fill(t, tc, c->n_inst, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return RTBTE_OK;
}

extern "C" int rtbte_get_stats(const rtbte_ctx* c, int32_t inst, rtbte_stats* out) {
  if (!c || !out || inst < 0 || inst >= c->n_inst) return RTBTE_E_INVAL;
  InstState s, f, w;
  int32_t health = 0;
  if (hipSetDevice(c->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(&s, c->st + inst, sizeof s, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&f, c->st_fast + inst, sizeof f, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&w, c->st_slow, sizeof w, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&health, c->health + inst, sizeof health, hipMemcpyDeviceToHost) != hipSuccess)
    return RTBTE_E_HIP;
  std::memset(out, 0, sizeof *out);
  // ERK steps, plus MIS slow steps (fixed and adaptive; common to a batch)
  out->n_accept = s.n_accept + c->slow_steps + w.n_accept;
  out->n_reject = s.n_reject + w.n_reject;
  out->n_fast_accept = f.n_accept;
  out->n_fast_reject = f.n_reject;
  const int64_t main_evals = s.n_evals, fast_evals = f.n_evals;
  // the fast state also ran the slow sub-flows of splitting steps
  out->n_rhs_eph = main_evals + fast_evals - c->split_slow_evals + c->extra_rhs[0];
  out->n_rhs_phe = main_evals + fast_evals - c->split_slow_evals + c->extra_rhs[1];
  out->n_rhs_phph = main_evals + c->split_slow_evals + c->extra_rhs[2];
  out->t = s.t;
  out->h_last = s.h;
  out->h_min = s.h_min;
  out->h_max = s.h_max;
  out->eps_last = s.eps;
  out->err_vs_fp64_last = c->err64[(size_t)inst];
  out->status = c->last_status;
  out->health = health;
  return RTBTE_OK;
}

extern "C" int rtbte_get_state(const rtbte_ctx* c, void* buf, size_t* len) {
  if (!c || !len) return RTBTE_E_INVAL;
  const size_t ns = (2 * (size_t)c->n_inst + 1) * sizeof(InstState);
  const size_t need = ns + 5 * sizeof(int64_t) + (size_t)c->n_inst * sizeof(int32_t);
  if (!buf) {
    *len = need;
    return RTBTE_OK;
  }
  if (*len < need) return RTBTE_E_INVAL;
  char* p = (char*)buf;
  if (hipSetDevice(c->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(p, c->st, c->n_inst * sizeof(InstState), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(p + c->n_inst * sizeof(InstState), c->st_fast, c->n_inst * sizeof(InstState),
                hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(p + 2 * c->n_inst * sizeof(InstState), c->st_slow, sizeof(InstState), hipMemcpyDeviceToHost) !=
          hipSuccess ||
      hipMemcpy(p + ns + 5 * sizeof(int64_t), c->health, (size_t)c->n_inst * sizeof(int32_t),
                hipMemcpyDeviceToHost) != hipSuccess)
    return RTBTE_E_HIP;
  int64_t tail[5] = {c->extra_rhs[0], c->extra_rhs[1], c->extra_rhs[2], c->slow_steps, c->split_slow_evals};
  std::memcpy(p + ns, tail, sizeof tail);
  *len = need;
  return RTBTE_OK;
}

extern "C" int rtbte_set_state(rtbte_ctx* c, const void* buf, size_t len) {
  if (!c || !buf) return RTBTE_E_INVAL;
  const size_t ns = (2 * (size_t)c->n_inst + 1) * sizeof(InstState);
  const size_t need = ns + 5 * sizeof(int64_t) + (size_t)c->n_inst * sizeof(int32_t);
  if (len != need) return fail(c, RTBTE_E_INVAL, "state size %zu, expected %zu", len, need);
  const char* p = (const char*)buf;
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipMemcpy(c->st, p, c->n_inst * sizeof(InstState), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->st_fast, p + c->n_inst * sizeof(InstState), c->n_inst * sizeof(InstState),
                      hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->st_slow, p + 2 * c->n_inst * sizeof(InstState), sizeof(InstState),
                      hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->health, p + ns + 5 * sizeof(int64_t), (size_t)c->n_inst * sizeof(int32_t),
                      hipMemcpyHostToDevice));
  int64_t tail[5];
  std::memcpy(tail, p + ns, sizeof tail);
  c->extra_rhs[0] = tail[0];
  c->extra_rhs[1] = tail[1];
  c->extra_rhs[2] = tail[2];
  c->slow_steps = tail[3];
  c->split_slow_evals = tail[4];
  return RTBTE_OK;
}

extern "C" int rtbte_profile(rtbte_ctx* c, int32_t enable) {
  if (!c) return RTBTE_E_INVAL;
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipDeviceSynchronize());
  HIPCHK(c, harvest(c));
  c->prof = enable != 0;
  c->prof_ms = 0.0;
  c->prof_bytes = 0.0;
  c->prof_n = 0;
  return RTBTE_OK;
}

extern "C" int rtbte_profile_read(rtbte_ctx* c, double* total_ms, int64_t* launches, double* bytes) {
  if (!c) return RTBTE_E_INVAL;
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipDeviceSynchronize());
  HIPCHK(c, harvest(c));
  if (total_ms) *total_ms = c->prof_ms;
  if (launches) *launches = c->prof_n;
  if (bytes) *bytes = c->prof_bytes;
  return RTBTE_OK;
}

// ------------------------------------------------------------------ autotuner
namespace {

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}

// Cache key: device, precision and weight format, and the sizes and
// parameters of every instance.  A collision can only cost speed: every
// launch shape gives the same results to rounding order.
std::string tune_key(const rtbte_problem* P, int n, const rtbte_options& o) {
  hipDeviceProp_t prop{};
  (void)hipGetDeviceProperties(&prop, o.device);
  uint64_t h = 1469598103934665603ull;
  h = fnv1a(h, &n, sizeof n);
  for (int i = 0; i < n; ++i) {
    const rtbte_problem& p = P[i];
    const int64_t v[6] = {p.n_el, p.n_ph, p.n_k_total, p.n_q_total, p.n_eph, p.n_pp};
    const double d[4] = {p.sigma_eph, p.sigma_pp, p.nsigma, p.hw_cut};
    h = fnv1a(h, v, sizeof v);
    h = fnv1a(h, d, sizeof d);
  }
  const int32_t f[2] = {o.precision, o.precision == RTBTE_MIXED ? o.mixed_weights : 0};
  h = fnv1a(h, f, sizeof f);
  char buf[160];
  snprintf(buf, sizeof buf, "%s-cu%d-%016llx", prop.gcnArchName, prop.multiProcessorCount,
           (unsigned long long)h);
  for (char* q = buf; *q; ++q)
    if (*q == ' ' || *q == ':') *q = '_';
  return buf;
}

// Cache file: one line per entry, "key rows_el rows_ph item_channels ms";
// the last line with the key wins.
bool cache_lookup(const char* path, const std::string& key, int* ge, int* gp, int64_t* ich) {
  if (!path || !*path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char k[200];
  int a, b;
  long long ic;
  double ms;
  bool hit = false;
  while (fscanf(f, "%199s %d %d %lld %lf", k, &a, &b, &ic, &ms) == 5)
    if (key == k && valid_group_rows(a) && valid_group_rows(b) && ic > 0) {
      *ge = a; *gp = b; *ich = ic; hit = true;
    }
  fclose(f);
  return hit;
}

void cache_store(const char* path, const std::string& key, int ge, int gp, int64_t ich, double ms) {
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %d %d %lld %.6f\n", key.c_str(), ge, gp, (long long)ich, ms);
  fclose(f);
}

// Mean time of one full right-hand side (collision kernel and row fix-up)
// over `reps` launches after two untimed ones, on a stream of its own.
int time_rhs(rtbte_ctx* c, const double* y, double* ydot, int reps, double* ms) {
  hipStream_t s = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  HIPCHK(c, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  FinishArgs f{};
  f.out = ydot;
  for (int i = 0; i < 2 && e == hipSuccess; ++i) e = rhs_launch(c, y, RTBTE_PART_ALL, nullptr, f, false, s);
  if (e == hipSuccess) e = hipEventRecord(a, s);
  for (int i = 0; i < reps && e == hipSuccess; ++i) e = rhs_launch(c, y, RTBTE_PART_ALL, nullptr, f, false, s);
  if (e == hipSuccess) e = hipEventRecord(b, s);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipStreamDestroy(s);
  if (e != hipSuccess) return fail(c, RTBTE_E_HIP, "tuning: %s", hipGetErrorString(e));
  *ms = (double)t / reps;
  return RTBTE_OK;
}

// Coordinate search over launch shapes: rows per group (each candidate is a
// full channel layout) and, for each layout, channels per work item (only the
// item table is rebuilt).  The fastest context is kept, a later candidate
// replacing the one kept only when it is faster by more than kTuneMargin
// (the spread of repeated timings), so that the choice does not flip between
// runs on noise; the shape goes to the cache file.
constexpr double kTuneMargin = 0.02;
constexpr int kTuneReps = 20;
int tune_create(const rtbte_problem* P, int n, rtbte_options o, rtbte_ctx** out) {
  const char* path = o.tune_cache ? o.tune_cache : getenv("RTBTE_TUNE_CACHE");
  if (hipSetDevice(o.device) != hipSuccess) return fail(nullptr, RTBTE_E_HIP, "hipSetDevice failed");
  const std::string key = tune_key(P, n, o);
  o.tune = 0;
  int ge = 0, gp = 0;
  int64_t ich = 0;
  if (cache_lookup(path, key, &ge, &gp, &ich)) {
    o.group_rows_el = ge;
    o.group_rows_ph = gp;
    o.item_channels = ich;
    const int rc = create_impl(P, n, &o, out);
    if (rc == RTBTE_OK) (*out)->tuned = 2;
    return rc;
  }
  const int ge0 = o.group_rows_el ? o.group_rows_el : 8, gp0 = o.group_rows_ph ? o.group_rows_ph : 16;
  std::vector<std::pair<int, int>> layouts = {{ge0, gp0}, {4, gp0}, {16, gp0}, {ge0, 8}};
  rtbte_ctx* best = nullptr;
  double best_ms = INFINITY;
  int64_t best_ich = 0;
  double* y = nullptr;
  double* yd = nullptr;
  std::vector<std::pair<int, int>> seen;
  int rc = RTBTE_OK;
  for (auto lay : layouts) {
    if (std::find(seen.begin(), seen.end(), lay) != seen.end()) continue;
    seen.push_back(lay);
    rtbte_options oc = o;
    oc.group_rows_el = lay.first;
    oc.group_rows_ph = lay.second;
    oc.item_channels = 0;
    rtbte_ctx* c = nullptr;
    rc = create_impl(P, n, &oc, &c);
    if (rc == RTBTE_E_NOMEM && best) {  // a second layout does not fit beside the best one
      rc = RTBTE_OK;
      continue;
    }
    if (rc != RTBTE_OK) break;
    if (!y) {
      hipError_t e = hipMalloc((void**)&y, (size_t)std::max<int64_t>(c->ny, 1) * sizeof(double));
      if (e == hipSuccess) e = hipMalloc((void**)&yd, (size_t)std::max<int64_t>(c->ny, 1) * sizeof(double));
      if (e == hipSuccess) e = hipMemset(y, 0, (size_t)std::max<int64_t>(c->ny, 1) * sizeof(double));
      if (e != hipSuccess) {
        rtbte_destroy(c);
        rc = fail(nullptr, RTBTE_E_NOMEM, "tuning buffers: %s", hipGetErrorString(e));
        break;
      }
    }
    const int64_t base = o.item_channels > 0 ? o.item_channels : c->item_channels;
    std::vector<int64_t> cand = {base, std::max<int64_t>(512, base / 2), std::min<int64_t>(1 << 20, base * 2)};
    double c_best = INFINITY;
    int64_t c_ich = 0;
    std::vector<int64_t> tried;
    for (int64_t ic : cand) {
      if (std::find(tried.begin(), tried.end(), ic) != tried.end()) continue;
      tried.push_back(ic);
      if (ic != c->item_channels && rebuild_items(c, ic) != hipSuccess) {
        rc = fail(nullptr, RTBTE_E_NOMEM, "tuning: work items");
        break;
      }
      double ms = 0.0;
      rc = time_rhs(c, y, yd, kTuneReps, &ms);
      if (rc != RTBTE_OK) {
        g_create_error = c->err;
        break;
      }
      if (ms < c_best * (1.0 - kTuneMargin)) { c_best = ms; c_ich = ic; }
    }
    if (rc != RTBTE_OK) {
      rtbte_destroy(c);
      break;
    }
    if (c_best < best_ms * (1.0 - kTuneMargin)) {
      if (c->item_channels != c_ich && rebuild_items(c, c_ich) != hipSuccess) {
        rtbte_destroy(c);
        rc = fail(nullptr, RTBTE_E_NOMEM, "tuning: work items");
        break;
      }
      if (best) rtbte_destroy(best);
      best = c;
      best_ms = c_best;
      best_ich = c_ich;
    } else {
      rtbte_destroy(c);
    }
  }
  if (y) (void)hipFree(y);
  if (yd) (void)hipFree(yd);
  if (rc != RTBTE_OK) {
    if (best) rtbte_destroy(best);
    return rc;
  }
  best->tuned = 1;
  best->tuned_ms = best_ms;
  best->opt.tune = 1;
  if (rtbte_reset(best) != RTBTE_OK) {
    const std::string msg = best->err;
    rtbte_destroy(best);
    return fail(nullptr, RTBTE_E_HIP, "%s", msg.c_str());
  }
  cache_store(path, key, best->group_rows_el, best->group_rows_ph, best_ich, best_ms);
  *out = best;
  return RTBTE_OK;
}

}  // namespace

extern "C" int rtbte_create(const rtbte_problem* problems, int32_t n_inst, const rtbte_options* opts,
                            rtbte_ctx** out) {
  TraceRange tr("rtbte_create");
  g_create_error.clear();
  if (!out) return fail(nullptr, RTBTE_E_INVAL, "out is NULL");
  *out = nullptr;
  rtbte_options o;
  if (opts) o = *opts;
  else rtbte_default_options(&o);
  if (o.tune) {
    // the candidate contexts check every argument themselves
    return tune_create(problems, n_inst, o, out);
  }
  return create_impl(problems, n_inst, &o, out);
}

// ---------------------------------------------------------------- observables
namespace {

// Upload a CSR (ptr[n+1], idx) built on the host, run `body`, free it.
template <class F>
int with_csr(rtbte_ctx* c, const std::vector<int32_t>& ptr, const std::vector<int32_t>& idx, hipStream_t s,
             F&& body) {
  int32_t *dp = nullptr, *di = nullptr;
  hipError_t e = upload(&dp, ptr.data(), ptr.size());
  if (e == hipSuccess) e = upload(&di, idx.empty() ? ptr.data() : idx.data(), std::max<size_t>(idx.size(), 1));
  int rc = e == hipSuccess ? body(dp, di) : fail(c, RTBTE_E_NOMEM, "observables: %s", hipGetErrorString(e));
  if (rc == RTBTE_OK) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = fail(c, RTBTE_E_HIP, "observables: %s", hipGetErrorString(e));
  }
  if (dp) (void)hipFree(dp);
  if (di) (void)hipFree(di);
  return rc;
}

}  // namespace

extern "C" int rtbte_energy_average(rtbte_ctx* c, const double* y, const double* y_ref, int32_t inst,
                                    int32_t which, double e_lo, double e_hi, int32_t n_bins, double* out,
                                    void* stream) {
  if (!c) return RTBTE_E_INVAL;
  if (!y || !out || inst < 0 || inst >= c->n_inst || (which != 0 && which != 1) || n_bins < 1 ||
      !(e_hi > e_lo))
    return fail(c, RTBTE_E_INVAL, "rtbte_energy_average: bad arguments");
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  const InstInfo& in = c->info[inst];
  const int64_t b0 = in.off + (which ? in.n_el : 0), n = which ? in.n_ph : in.n_el;
  // states by bin (stable counting sort), bins [e_lo + k de, e_lo + (k+1) de)
  std::vector<int32_t> ptr((size_t)n_bins + 1, 0), bin((size_t)n);
  const double de = (e_hi - e_lo) / n_bins;
  for (int64_t j = 0; j < n; ++j) {
    const double x = c->energy_h[(size_t)(b0 + j)];
    int32_t k = -1;
    if (x >= e_lo && x < e_hi) k = std::min<int32_t>(n_bins - 1, (int32_t)std::floor((x - e_lo) / de));
    bin[(size_t)j] = k;
    if (k >= 0) ptr[(size_t)k + 1]++;
  }
  for (int k = 0; k < n_bins; ++k) ptr[(size_t)k + 1] += ptr[(size_t)k];
  std::vector<int32_t> idx((size_t)ptr[(size_t)n_bins]), cur(ptr.begin(), ptr.end() - 1);
  for (int64_t j = 0; j < n; ++j)
    if (bin[(size_t)j] >= 0) idx[(size_t)cur[(size_t)bin[(size_t)j]]++] = (int32_t)(b0 + j);
  double* dout = nullptr;
  HIPCHK(c, hipMalloc((void**)&dout, 3 * (size_t)n_bins * sizeof(double)));
  int rc = with_csr(c, ptr, idx, s, [&](int32_t* dp, int32_t* di) -> int {
    HIPCHK(c, launch_bin_means(y, y_ref, di, dp, n_bins, dout, s));
    HIPCHK(c, hipMemcpyAsync(out, dout, 3 * (size_t)n_bins * sizeof(double), hipMemcpyDeviceToHost, s));
    return RTBTE_OK;
  });
  (void)hipFree(dout);
  return rc;
}

extern "C" int rtbte_mode_temperatures(rtbte_ctx* c, const double* y, int32_t inst, const int32_t* mode_of,
                                       int32_t n_modes, double* T_out, void* stream) {
  if (!c) return RTBTE_E_INVAL;
  if (!y || !mode_of || !T_out || inst < 0 || inst >= c->n_inst || n_modes < 1)
    return fail(c, RTBTE_E_INVAL, "rtbte_mode_temperatures: bad arguments");
  const InstInfo& in = c->info[inst];
  for (int32_t j = 0; j < in.n_ph; ++j)
    if (mode_of[j] < 0 || mode_of[j] >= n_modes)
      return fail(c, RTBTE_E_INVAL, "rtbte_mode_temperatures: mode_of[%d] = %d out of range", j, mode_of[j]);
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  std::vector<int32_t> ptr((size_t)n_modes + 1, 0), idx((size_t)in.n_ph);
  for (int32_t j = 0; j < in.n_ph; ++j) ptr[(size_t)mode_of[j] + 1]++;
  for (int k = 0; k < n_modes; ++k) ptr[(size_t)k + 1] += ptr[(size_t)k];
  std::vector<int32_t> cur(ptr.begin(), ptr.end() - 1);
  for (int32_t j = 0; j < in.n_ph; ++j) idx[(size_t)cur[(size_t)mode_of[j]]++] = (int32_t)(in.off + in.n_el + j);
  double* dT = nullptr;
  HIPCHK(c, hipMalloc((void**)&dT, (size_t)n_modes * sizeof(double)));
  int rc = with_csr(c, ptr, idx, s, [&](int32_t* dp, int32_t* di) -> int {
    HIPCHK(c, launch_mode_temperature(y, c->energy_d, di, dp, n_modes, dT, s));
    HIPCHK(c, hipMemcpyAsync(T_out, dT, (size_t)n_modes * sizeof(double), hipMemcpyDeviceToHost, s));
    return RTBTE_OK;
  });
  (void)hipFree(dT);
  return rc;
}
