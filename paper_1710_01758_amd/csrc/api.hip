// Host side of libpics.so: context, validation, workspace and the
// orchestration of the kernels behind the C ABI declared in include/pics.h.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <sys/stat.h>
#include <unistd.h>
#include <string>
#include <vector>

#include "pics.h"
#include "fft.hpp"
#include "internal.hpp"
#include "learned.hpp"

using namespace pics;

struct pics_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int nslices = 0;
  std::vector<pics_desc> desc;
  std::vector<SliceDev> sl;
  long long img_total = 0, coil_total = 0, mask_total = 0, aux_total = 0, max_pixels = 0;
  int max_levels = 0;
  bool any_wavelet = false, any_nowavelet = false, any_2d = false;
  std::vector<int> wave_tiles;  // per level: max over slices of 16 x 16 coefficient tiles

  struct Group {
    int m, n;
    std::vector<int> idx;
    int* idx_dev;
    int coil_groups = 1;  // workgroups sharing one tile's coil loop (autotuned)
    int tile = 0;         // column-tile width of the line-mask operator (autotuned; 0 = col_tile(m))
    int nc_max = 0;
    int sidx = 0;         // index of the group's side stream
    int mask_kind = 0;    // PICS_MASK_LINES or PICS_MASK_2D (slices of one group share it)
  };
  std::vector<Group> groups;
  int* all_idx_dev = nullptr;

  const float2* sens = nullptr;
  const uint8_t* masks = nullptr;

  // one device block for everything the context owns
  void* block = nullptr;
  SliceDev* sl_dev = nullptr;
  float2* tw = nullptr;
  float2 *r, *t, *z, *p, *pn, *q, *g1, *g, *rhs, *bx, *by, *bx2, *by2, *bw, *ux, *uy, *uw, *w1, *w2;
  float2* coiltmp = nullptr;
  float *kraw, *kinv, *jac, *ftmp;
  double *part, *pbar;
  PcgState* st = nullptr;
  int* bad = nullptr;
  // iteration-lock schedule and per-solve history, sized for `solves_cap`
  // solves: inside `block` as created, in `reserve_block` once pics_reserve
  // has enlarged them
  long long solves_cap = 0;
  int* lock_dev = nullptr;       // [solves_cap][nslices]
  long long lock_cap = 0;        // ints at lock_dev
  void* reserve_block = nullptr;

  PcgState* st_host = nullptr;  // pinned
  int* flag_host = nullptr;      // pinned
  int pk = PK_NONE;
  int poll_chunk = 2;
  std::string err;

  // Split Bregman outer iterations replayed from a captured graph
  int graph_budget = 1;          // PCG iterations per solve inside the graph (0: host-polled only)
  int graph_first_budget = 8;    // the same for the first solve (from the root-sum-of-squares start)
  int* solve_counter = nullptr;  // device: history row of the next solve
  int* hist = nullptr;           // device: [solves][nslices] iterations, then [solves][nslices] status
  long long hist_cap = 0;        // ints at hist (2 solves_cap nslices)
  std::vector<int> hist_host;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  struct GraphKey {
    const void* x;
    const void* kspace;
    double tol;
    int budget, first_budget, pk, n_inner, n_rep;
    const int* hist;
    int tuning;  // tuning generation: a new coil split or workspace needs a new graph
    bool operator==(const GraphKey& o) const {
      return x == o.x && kspace == o.kspace && tol == o.tol && budget == o.budget &&
             first_budget == o.first_budget && pk == o.pk && n_inner == o.n_inner && n_rep == o.n_rep &&
             hist == o.hist && tuning == o.tuning;
    }
  } graph_key{};
  int graph_fallbacks = 0;       // solves that exceeded the budget (reconstruction redone host-polled)

  // Size groups touch disjoint slices, so their per-group kernels run on side
  // streams, forked from and joined back to the context's stream with events.
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> side_done;
  hipEvent_t fork_ev = nullptr;
  int forked = 0;
  bool concurrent_groups = true;

  float2* dpart = nullptr;       // per-coil-group partial data terms [groups][image-packed]
  int dpart_groups = 0;
  float2* scratch_dev = nullptr; // device address of `scratch` on this context's GPU (apply_A_noalloc)
  int tuning_gen = 0;            // bumped whenever a coil split or dpart changes
};

// Scratch of apply_A_noalloc, for callers that cannot allocate: the coil
// groups' partial data terms.  Every GPU that loads the library holds its own
// copy until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: kernels and copies take the per-device
// address that scratch_address() resolves, never the array's name.
static __device__ __align__(256) float2 scratch[PICS_NOALLOC_SCRATCH_BYTES / sizeof(float2)];

namespace {

constexpr int kMaxDevices = 64;
constexpr long long kDefaultSolves = 64;  // solves per reconstruction reserved by pics_create
std::mutex g_scratch_mu;
float2* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be current: looked up
// once per device, then served from the table.
hipError_t scratch_address(int device, float2** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_addr[device] = (float2*)p;
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}

}  // namespace

namespace {

int fail(pics_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIPCHK(ctx, expr)                                                                          \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) return fail(ctx, PICS_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

Ws make_ws(const pics_ctx* c) {
  Ws w;
  w.sl = c->sl_dev;
  w.group = c->all_idx_dev;
  w.sens = c->sens;
  w.mask = c->masks;
  w.tw = c->tw;
  w.kinv = c->kinv;
  w.jac = c->jac;
  w.part = c->part;
  w.st = c->st;
  return w;
}

Launch make_launch(const pics_ctx* c, const pics_ctx::Group& g) {
  Launch L;
  L.stream = c->forked ? c->side[g.sidx] : c->stream;
  L.m = g.m;
  L.n = g.n;
  L.count = (int)g.idx.size();
  L.group = g.idx_dev;
  return L;
}

Simple make_simple(const pics_ctx* c) {
  Simple S;
  S.stream = c->stream;
  S.nslices = c->nslices;
  S.max_pixels = c->max_pixels;
  return S;
}

// Scope in which make_launch hands each size group its side stream: the
// side streams wait for the work already on the context's stream, and the
// context's stream waits for all of them when the scope ends.  Works under
// stream capture (the side streams join the capture through the events).
struct GroupFork {
  pics_ctx* c;
  bool on = false;
  hipError_t err = hipSuccess;
  explicit GroupFork(pics_ctx* cc) : c(cc) {
    if (c->side.empty() || !c->concurrent_groups || c->forked) return;
    err = hipEventRecord(c->fork_ev, c->stream);
    for (size_t i = 0; i < c->side.size() && err == hipSuccess; ++i) err = hipStreamWaitEvent(c->side[i], c->fork_ev, 0);
    on = err == hipSuccess;
    c->forked = on;
  }
  hipError_t join() {
    if (!on) return err;
    on = false;
    c->forked = 0;
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < c->side.size(); ++i) {
      hipError_t e1 = hipEventRecord(c->side_done[i], c->side[i]);
      if (e1 == hipSuccess) e1 = hipStreamWaitEvent(c->stream, c->side_done[i], 0);
      if (e == hipSuccess) e = e1;
    }
    return e;
  }
  ~GroupFork() { (void)join(); }
};

// Ws whose group table is the group's slice list (grid.y -> slice)
Ws ws_for(const pics_ctx* c, const pics_ctx::Group& g) {
  Ws w = make_ws(c);
  w.group = g.idx_dev;
  return w;
}

// The system operator on one size group: the fused column-tile kernel for
// line masks, the three-pass 2D-transform path for 2D masks.
// split, dpart: coil split of the line-mask kernel and the buffer of its
// partial sums (split 0: the group's tuned split and the context's table).
hipError_t launch_operator(pics_ctx* c, const pics_ctx::Group& g, int mode, int terms, int pk, double tol,
                           const float2* xin, const float2* zsrc, const float2* pold, float2* pn, float2* out,
                           int split = 0, float2* dpart = nullptr) {
  if (g.mask_kind == PICS_MASK_2D)
    return launch_apply2d(make_launch(c, g), ws_for(c, g), mode, terms, pk, tol, xin, zsrc, pold, pn, out,
                          c->coiltmp);
  if (split == 0) {
    split = g.coil_groups;
    dpart = c->dpart;
  }
  // a coil split runs with the default tiles (the tuner never pairs the two)
  const int tile = split > 1 ? 0 : g.tile;
  return launch_col_apply(make_launch(c, g), ws_for(c, g), mode, terms, pk, tol, xin, zsrc, pold, pn, out, split,
                          dpart, c->img_total, tile, g.nc_max);
}

}  // namespace

// twiddles tw[k] = exp(-2 pi i k / N), computed in double
void pics::fill_twiddles(float2* tw) {
  for (int N : kSupportedSizes) {
    const int off = tw_offset(N);
    for (int k = 0; k < N; ++k) {
      const double a = -2.0 * M_PI * (double)k / (double)N;
      tw[off + k] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
  }
}

namespace {

bool levels_ok(int m, int n, int levels) {
  for (int l = 0; l < levels; ++l) {
    if ((m >> l) % 2 || (n >> l) % 2 || (m >> l) < 2 || (n >> l) < 2) return false;
  }
  return true;
}

bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

// W (all levels).  Level l reads `in` (l = 0) or the approximation block the
// previous level left in the ping-pong buffers, and writes its own
// approximation block to w1 (l even) or w2 (l odd); final coefficients go to
// `coef` (mode 0) or through the shrink/update into bw / uw (mode 1).
int wavelet_analysis(pics_ctx* c, const float2* in, int mode, float2* coef, float2* bw, float2* uw, const TvArgs& tv) {
  const Ws w = make_ws(c);
  const Simple S = make_simple(c);
  for (int l = 0; l < c->max_levels; ++l) {
    WaveArgs a{};
    a.level = l;
    a.inverse = 0;
    a.mode = mode;
    a.fresh = tv.fresh;
    a.in = l == 0 ? in : ((l - 1) % 2 == 0 ? c->w1 : c->w2);
    a.out = l % 2 == 0 ? c->w1 : c->w2;
    a.coef = coef;
    a.bw = bw;
    a.uw = uw;
    TvArgs t = tv;
    t.enabled = (l == 0) ? tv.enabled : 0;
    if (l > 0) t.outer.rec = SolveRecord{};
    const hipError_t e = launch_wavelet(S, w, a, t, c->wave_tiles[l]);
    if (e != hipSuccess) return fail(c, PICS_ERR_HIP, "wavelet analysis: %s", hipGetErrorString(e));
  }
  return PICS_OK;
}

// W^H (all levels), coarsest first.  Mode 0 writes the image to `out`;
// mode 1 writes the Split Bregman right-hand side tvr + gam W^H coef into
// rhs, tvr = g + lam (D_x^H u_x + D_y^H u_y) as the level-0 analysis left it.
int wavelet_synthesis(pics_ctx* c, const float2* coef, int mode, float2* out, const float2* tvr, float2* rhs) {
  const Ws w = make_ws(c);
  const Simple S = make_simple(c);
  const int L = c->max_levels;
  auto buf = [&](int l) { return ((L - 1 - l) % 2 == 0) ? c->w1 : c->w2; };
  for (int l = L - 1; l >= 0; --l) {
    WaveArgs a{};
    a.level = l;
    a.inverse = 1;
    a.mode = mode;
    a.in = l + 1 < L ? buf(l + 1) : nullptr;
    a.out = l == 0 ? out : buf(l);
    a.coef = const_cast<float2*>(coef);
    a.tvr = tvr;
    a.rhs = rhs;
    TvArgs t{};
    const hipError_t e = launch_wavelet(S, w, a, t, c->wave_tiles[l]);
    if (e != hipSuccess) return fail(c, PICS_ERR_HIP, "wavelet synthesis: %s", hipGetErrorString(e));
  }
  return PICS_OK;
}

}  // namespace

// =====================================================================
extern "C" {

const char* pics_status_string(int s) {
  switch (s) {
    case PICS_OK: return "ok";
    case PICS_WARN_MAXIT: return "warning: PCG reached maxit";
    case PICS_WARN_FALLBACK: return "warning: learned spectrum rejected, circulant used";
    case PICS_ERR_INVALID: return "invalid argument";
    case PICS_ERR_UNSUPPORTED: return "unsupported size or mode";
    case PICS_ERR_NONFINITE: return "non-finite value in PCG";
    case PICS_ERR_BREAKDOWN: return "PCG breakdown (p^H A p <= 0)";
    case PICS_ERR_NOT_POSITIVE: return "circulant spectrum not positive";
    case PICS_ERR_HIP: return "HIP runtime error";
    case PICS_ERR_STATE: return "preconditioner not built";
    default: return "unknown status";
  }
}

const char* pics_last_error(const pics_ctx* c) { return c ? c->err.c_str() : "null context"; }

namespace {
int ensure_dpart(pics_ctx* c, int groups);

// Column-tile width of a group's line-mask operator; the slices' sigma
// partial count (one per tile) follows it on the host and device tables.
int set_group_tile(pics_ctx* c, pics_ctx::Group& g, int tile) {
  if (tile == col_tile(g.m)) tile = 0;
  if (tile == g.tile) return PICS_OK;
  g.tile = tile;
  const int ct = g.n / (tile ? tile : col_tile(g.m));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int s : g.idx) {
    c->sl[s].ctiles = ct;
    HIPCHK(c, hipMemcpy(c->sl_dev + s, &c->sl[s], sizeof(SliceDev), hipMemcpyHostToDevice));
  }
  ++c->tuning_gen;
  return PICS_OK;
}
}  // namespace

int pics_set_option(pics_ctx* c, int32_t key, int64_t value) {
  if (!c) return PICS_ERR_INVALID;
  if (key == PICS_OPT_POLL_CHUNK) {
    if (value < 1 || value > 1024) return fail(c, PICS_ERR_INVALID, "poll chunk out of range");
    c->poll_chunk = (int)value;
    return PICS_OK;
  }
  if (key == PICS_OPT_GRAPH_BUDGET) {
    if (value < 0 || value > 64) return fail(c, PICS_ERR_INVALID, "graph budget out of range");
    c->graph_budget = (int)value;
    return PICS_OK;
  }
  if (key == PICS_OPT_GRAPH_FIRST_BUDGET) {
    if (value < 1 || value > 256) return fail(c, PICS_ERR_INVALID, "first-solve graph budget out of range");
    c->graph_first_budget = (int)value;
    return PICS_OK;
  }
  if (key == PICS_OPT_CONCURRENT_GROUPS) {
    if (value < 0 || value > 1) return fail(c, PICS_ERR_INVALID, "concurrent groups: 0 or 1");
    c->concurrent_groups = value != 0;
    ++c->tuning_gen;
    return PICS_OK;
  }
  if (key == PICS_OPT_COIL_GROUPS) {
    if (value < 1 || value > 64) return fail(c, PICS_ERR_INVALID, "coil split out of range");
    int need = 1;
    for (auto& g : c->groups) need = std::max(need, std::min((int)value, g.nc_max));
    int rc = ensure_dpart(c, need);
    if (rc) return rc;
    for (auto& g : c->groups) {
      g.coil_groups = std::min((int)value, g.nc_max);
      if (g.coil_groups > 1 && (rc = set_group_tile(c, g, 0))) return rc;
    }
    ++c->tuning_gen;
    return PICS_OK;
  }
  if (key == PICS_OPT_COL_TILE) {
    for (auto& g : c->groups) {
      if (g.mask_kind != PICS_MASK_LINES) continue;
      const int tile = value == 0 ? col_tile(g.m) : (int)value;
      if (value < 0 || value > 64 || !apply_tile_ok(g.m, g.n, tile))
        return fail(c, PICS_ERR_INVALID, "column tile %lld not available for %d x %d slices", (long long)value, g.m,
                    g.n);
    }
    for (auto& g : c->groups) {
      if (g.mask_kind != PICS_MASK_LINES) continue;
      const int rc = set_group_tile(c, g, value == 0 ? 0 : (int)value);
      if (rc) return rc;
      if (value != 0) g.coil_groups = 1;
    }
    ++c->tuning_gen;
    return PICS_OK;
  }
  return fail(c, PICS_ERR_INVALID, "unknown option %d", key);
}

int pics_sizes(const pics_ctx* c, int64_t* img, int64_t* coil, int64_t* mask) {
  if (!c) return PICS_ERR_INVALID;
  if (img) *img = c->img_total;
  if (coil) *coil = c->coil_total;
  if (mask) *mask = c->mask_total;
  return PICS_OK;
}

int pics_reserve(pics_ctx* c, int32_t max_solves) {
  if (!c) return PICS_ERR_INVALID;
  if (max_solves < 1 || max_solves > (1 << 20)) return fail(c, PICS_ERR_INVALID, "pics_reserve: max_solves %d", max_solves);
  if (max_solves <= c->solves_cap) return PICS_OK;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const size_t lock_bytes = (sizeof(int) * (size_t)max_solves * c->nslices + 255) / 256 * 256;
  const size_t hist_bytes = sizeof(int) * 2 * (size_t)max_solves * c->nslices;
  void* blk = nullptr;
  HIPCHK(c, hipMalloc(&blk, lock_bytes + hist_bytes));
  if (c->graph_exec) {  // the graph records the old history's address
    (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
  }
  if (c->reserve_block) (void)hipFree(c->reserve_block);
  c->reserve_block = blk;
  c->solves_cap = max_solves;
  c->lock_dev = (int*)blk;
  c->lock_cap = (long long)max_solves * c->nslices;
  c->hist = (int*)((char*)blk + lock_bytes);
  c->hist_cap = 2LL * max_solves * c->nslices;
  return PICS_OK;
}

int pics_create(pics_ctx** out, int32_t nslices, const pics_desc* descs, const void* sens, const uint8_t* masks,
                void* stream) {
  if (!out) return PICS_ERR_INVALID;
  *out = nullptr;
  if (nslices < 1 || nslices > 65535 || !descs || !sens || !masks) return PICS_ERR_INVALID;
  for (int s = 0; s < nslices; ++s) {
    const pics_desc& d = descs[s];
    if (d.m <= 0 || d.n <= 0 || d.ncoils < 1 || d.ncoils > 4096) return PICS_ERR_INVALID;
    if (!finite_nonneg(d.mu) || !finite_nonneg(d.lambda) || !finite_nonneg(d.gamma)) return PICS_ERR_INVALID;
    if (d.wavelet < 0 || d.wavelet > 2 || d.levels < 0 || d.levels > 12) return PICS_ERR_INVALID;
    if (d.mask_kind != PICS_MASK_LINES && d.mask_kind != PICS_MASK_2D) return PICS_ERR_INVALID;
    if (!fft_size_supported(d.m) || !fft_size_supported(d.n)) return PICS_ERR_UNSUPPORTED;
    if (d.wavelet != PICS_WAVELET_NONE && !levels_ok(d.m, d.n, d.levels)) return PICS_ERR_UNSUPPORTED;
  }
  pics_ctx* c = new pics_ctx();
  c->nslices = nslices;
  c->stream = (hipStream_t)stream;
  c->sens = (const float2*)sens;
  c->masks = masks;
  c->desc.assign(descs, descs + nslices);
  if (hipGetDevice(&c->device) != hipSuccess || scratch_address(c->device, &c->scratch_dev) != hipSuccess) {
    delete c;
    return PICS_ERR_HIP;
  }

  std::map<std::tuple<int, int, int>, int> gidx;
  for (int s = 0; s < nslices; ++s) {
    const pics_desc& d = descs[s];
    SliceDev sd{};
    sd.m = d.m;
    sd.n = d.n;
    sd.nc = d.ncoils;
    sd.mask_kind = d.mask_kind;
    sd.wavelet = d.wavelet;
    sd.levels = d.wavelet == PICS_WAVELET_NONE ? 0 : d.levels;
    sd.mu = (float)d.mu;
    sd.lam = (float)d.lambda;
    sd.gam = (float)d.gamma;
    sd.ctiles = d.n / col_tile(d.m);
    sd.img = c->img_total;
    sd.coil = c->coil_total;
    sd.mask = c->mask_total;
    sd.aux = c->aux_total;
    const long long N = (long long)d.m * d.n;
    c->img_total += N;
    c->coil_total += N * d.ncoils;
    c->mask_total += d.mask_kind == PICS_MASK_LINES ? d.m : N;
    c->aux_total += (long long)(d.n / col_tile(d.m)) * d.m;
    c->max_pixels = std::max(c->max_pixels, N);
    c->max_levels = std::max(c->max_levels, sd.levels);
    if (d.mask_kind == PICS_MASK_2D) c->any_2d = true;
    if (sd.levels > 0) c->any_wavelet = true;
    else c->any_nowavelet = true;
    c->sl.push_back(sd);
    auto key = std::make_tuple(d.m, d.n, (int)d.mask_kind);
    auto it = gidx.find(key);
    if (it == gidx.end()) {
      gidx[key] = (int)c->groups.size();
      c->groups.push_back({d.m, d.n, {s}, nullptr});
      c->groups.back().nc_max = d.ncoils;
      c->groups.back().mask_kind = d.mask_kind;
    } else {
      c->groups[it->second].idx.push_back(s);
      c->groups[it->second].nc_max = std::max(c->groups[it->second].nc_max, (int)d.ncoils);
    }
  }

  c->wave_tiles.assign(c->max_levels, 0);
  for (int l = 0; l < c->max_levels; ++l)
    for (const SliceDev& sd : c->sl)
      if (sd.levels > l) c->wave_tiles[l] = std::max(c->wave_tiles[l], wavelet_tiles(sd.m, sd.n, l));

  // ---- one allocation for everything
  const long long I = c->img_total;
  std::vector<std::pair<void**, size_t>> plan;
  auto add = [&](void** ptr, size_t bytes) { plan.push_back({ptr, (bytes + 255) / 256 * 256}); };
  add((void**)&c->sl_dev, sizeof(SliceDev) * nslices);
  add((void**)&c->all_idx_dev, sizeof(int) * nslices);
  for (auto& g : c->groups) add((void**)&g.idx_dev, sizeof(int) * g.idx.size());
  add((void**)&c->tw, sizeof(float2) * kTwiddleTotal);
  float2** cbufs[] = {&c->r, &c->t, &c->z, &c->p, &c->pn, &c->q, &c->g1, &c->g, &c->rhs,
                      &c->bx, &c->by, &c->bx2, &c->by2, &c->bw, &c->ux, &c->uy, &c->uw, &c->w1, &c->w2};
  for (float2** b : cbufs) add((void**)b, sizeof(float2) * I);
  add((void**)&c->coiltmp, sizeof(float2) * c->coil_total);
  add((void**)&c->kraw, sizeof(float) * I);
  add((void**)&c->kinv, sizeof(float) * I);
  add((void**)&c->jac, sizeof(float) * I);
  add((void**)&c->ftmp, sizeof(float) * I);
  add((void**)&c->part, sizeof(double) * nslices * kSlots * kPartMax);
  add((void**)&c->pbar, sizeof(double) * std::max(1LL, c->aux_total));
  add((void**)&c->st, sizeof(PcgState) * nslices);
  add((void**)&c->bad, sizeof(int));
  add((void**)&c->solve_counter, sizeof(int));
  c->solves_cap = kDefaultSolves;
  c->lock_cap = kDefaultSolves * nslices;
  c->hist_cap = 2LL * kDefaultSolves * nslices;
  add((void**)&c->lock_dev, sizeof(int) * c->lock_cap);
  add((void**)&c->hist, sizeof(int) * c->hist_cap);
  size_t total = 0;
  for (auto& pr : plan) total += pr.second;
  if (hipMalloc(&c->block, total) != hipSuccess) {
    delete c;
    return PICS_ERR_HIP;
  }
  char* base = (char*)c->block;
  for (auto& pr : plan) {
    *pr.first = base;
    base += pr.second;
  }
  if (hipHostMalloc((void**)&c->st_host, sizeof(PcgState) * nslices, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->flag_host, sizeof(int) * 4, hipHostMallocDefault) != hipSuccess) {
    if (c->st_host) (void)hipHostFree(c->st_host);
    (void)hipFree(c->block);
    delete c;
    return PICS_ERR_HIP;
  }

  std::vector<float2> tw(kTwiddleTotal);
  fill_twiddles(tw.data());
  std::vector<int> all(nslices);
  for (int s = 0; s < nslices; ++s) all[s] = s;
  bool ok = hipMemcpy(c->tw, tw.data(), sizeof(float2) * kTwiddleTotal, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(c->sl_dev, c->sl.data(), sizeof(SliceDev) * nslices, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(c->all_idx_dev, all.data(), sizeof(int) * nslices, hipMemcpyHostToDevice) == hipSuccess;
  for (auto& g : c->groups)
    ok = ok && hipMemcpy(g.idx_dev, g.idx.data(), sizeof(int) * g.idx.size(), hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemset(c->part, 0, sizeof(double) * nslices * kSlots * kPartMax) == hipSuccess;
  if (ok && c->groups.size() > 1) {
    ok = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) == hipSuccess;
    for (size_t i = 0; i < c->groups.size() && ok; ++i) {
      hipStream_t st = nullptr;
      hipEvent_t ev = nullptr;
      ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
      if (st) c->side.push_back(st);
      if (ev) c->side_done.push_back(ev);
      c->groups[i].sidx = (int)i;
    }
  }
  if (!ok) {
    for (auto st : c->side) (void)hipStreamDestroy(st);
    for (auto ev : c->side_done) (void)hipEventDestroy(ev);
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    (void)hipHostFree(c->st_host);
    (void)hipHostFree(c->flag_host);
    (void)hipFree(c->block);
    delete c;
    return PICS_ERR_HIP;
  }
  *out = c;
  return PICS_OK;
}

int pics_destroy(pics_ctx* c) {
  if (!c) return PICS_ERR_INVALID;
  // best-effort release: errors are ignored on the way out
  (void)hipStreamSynchronize(c->stream);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->reserve_block) (void)hipFree(c->reserve_block);
  if (c->dpart) (void)hipFree(c->dpart);
  for (auto st : c->side) (void)hipStreamDestroy(st);
  for (auto ev : c->side_done) (void)hipEventDestroy(ev);
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  if (c->st_host) (void)hipHostFree(c->st_host);
  if (c->flag_host) (void)hipHostFree(c->flag_host);
  if (c->block) (void)hipFree(c->block);
  delete c;
  return PICS_OK;
}

int build_preconditioner(pics_ctx* c, int32_t kind, const float* correction, float* khat_out) {
  if (!c) return PICS_ERR_INVALID;
  if (kind < PICS_PRECOND_NONE || kind > PICS_PRECOND_LEARNED) return fail(c, PICS_ERR_INVALID, "kind %d", kind);
  if (kind == PICS_PRECOND_LEARNED && !correction) return fail(c, PICS_ERR_INVALID, "LEARNED needs a correction");
  if (kind == PICS_PRECOND_NONE) {
    c->pk = PK_NONE;
    return PICS_OK;
  }
  const Ws w = make_ws(c);
  int rc = PICS_OK;
  for (int attempt = 0; attempt < 2; ++attempt) {
    const float* corr = (kind == PICS_PRECOND_LEARNED && attempt == 0) ? correction : nullptr;
    {
      // line masks: axis-0 transforms of the coil maps give Pbar (and the
      // pixel coil energy in jac); 2D masks: full 2D transforms give P
      GroupFork fk(c);
      for (auto& g : c->groups) {
        if (g.mask_kind == PICS_MASK_2D) {
          HIPCHK(c, launch_row_fft(make_launch(c, g), ws_for(c, g), 0, 2, c->sens, c->coiltmp));
          HIPCHK(c, launch_col_power2d(make_launch(c, g), ws_for(c, g), c->coiltmp, c->ftmp, c->jac));
        } else {
          HIPCHK(c, launch_col_coil_power(make_launch(c, g), ws_for(c, g), c->pbar, c->jac));
        }
      }
      HIPCHK(c, fk.join());
    }
    HIPCHK(c, hipMemsetAsync(c->bad, 0, sizeof(int), c->stream));
    if (c->any_2d) {
      // 2D masks: k_c = IDFT(DFT(r) conj(DFT(P))) / N^3 (t, z, r, p as scratch)
      const Simple S = make_simple(c);
      HIPCHK(c, launch_corr_prep(S, w, c->ftmp, c->t, c->z));
      {
        GroupFork fk(c);
        for (auto& g : c->groups) {
          if (g.mask_kind != PICS_MASK_2D) continue;
          HIPCHK(c, launch_row_fft(make_launch(c, g), ws_for(c, g), 0, 0, c->t, c->r));
          HIPCHK(c, launch_col_fft(make_launch(c, g), ws_for(c, g), 0, c->r, c->t));
          HIPCHK(c, launch_row_fft(make_launch(c, g), ws_for(c, g), 0, 0, c->z, c->p));
          HIPCHK(c, launch_col_fft(make_launch(c, g), ws_for(c, g), 0, c->p, c->z));
        }
        HIPCHK(c, fk.join());
      }
      HIPCHK(c, launch_corr_mul(S, w, c->t, c->z));
      {
        GroupFork fk(c);
        for (auto& g : c->groups) {
          if (g.mask_kind != PICS_MASK_2D) continue;
          HIPCHK(c, launch_row_fft(make_launch(c, g), ws_for(c, g), 1, 0, c->t, c->r));
          HIPCHK(c, launch_col_fft(make_launch(c, g), ws_for(c, g), 1, c->r, c->t));
        }
        HIPCHK(c, fk.join());
      }
      HIPCHK(c, launch_build_k2d(S, w, c->t, corr, c->jac, c->kraw, c->kinv, c->jac, c->bad));
    }
    HIPCHK(c, launch_build_k(make_simple(c), w, c->pbar, corr, c->kraw, c->kinv, c->jac, c->bad));
    HIPCHK(c, hipMemcpyAsync(c->flag_host, c->bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (!c->flag_host[0]) break;
    if (kind != PICS_PRECOND_LEARNED || attempt == 1) {
      c->pk = PK_NONE;
      return fail(c, PICS_ERR_NOT_POSITIVE, "circulant spectrum has an entry <= 0 or not finite");
    }
    rc = PICS_WARN_FALLBACK;  // retry without the correction
    kind = PICS_PRECOND_CIRCULANT;
  }
  c->pk = kind;
  if (khat_out)
    HIPCHK(c, hipMemcpyAsync(khat_out, c->kraw, sizeof(float) * c->img_total, hipMemcpyDeviceToDevice, c->stream));
  return rc;
}

int apply_A(pics_ctx* c, const void* x, void* y, int32_t terms) {
  if (!c) return PICS_ERR_INVALID;
  if (!x || !y || x == y) return fail(c, PICS_ERR_INVALID, "apply_A: null or aliased buffers");
  if (terms < 0 || terms > (PICS_TERM_ALL | PICS_TERM_WAVELET_EXPLICIT))
    return fail(c, PICS_ERR_INVALID, "apply_A: terms %d", terms);
  const bool explicit_w = (terms & PICS_TERM_WAVELET_EXPLICIT) && (terms & PICS_TERM_GAMMA);
  const int kterms = explicit_w ? (terms & (TERM_DATA | TERM_TV)) : (terms & TERM_ALL);
  {
    GroupFork fk(c);
    for (auto& g : c->groups)
      HIPCHK(c, launch_operator(c, g, CA_APPLY, kterms, c->pk, 0.0, (const float2*)x, nullptr, nullptr, nullptr,
                                (float2*)y));
    HIPCHK(c, fk.join());
  }
  if (explicit_w) {
    // gam W^H W x through the wavelet kernels (coefficients in z, image in r)
    TvArgs none{};
    int rc = wavelet_analysis(c, (const float2*)x, 0, c->z, nullptr, nullptr, none);
    if (rc) return rc;
    rc = wavelet_synthesis(c, c->z, 0, c->r, nullptr, nullptr);
    if (rc) return rc;
    HIPCHK(c, launch_add_gamma(make_simple(c), make_ws(c), c->r, (const float2*)x, (float2*)y));
  }
  return PICS_OK;
}

int apply_A_noalloc(pics_ctx* c, const void* x, void* y, int32_t terms, int32_t coil_groups) {
  if (!c) return PICS_ERR_INVALID;
  if (!x || !y || x == y) return fail(c, PICS_ERR_INVALID, "apply_A_noalloc: null or aliased buffers");
  if (terms < 0 || terms > (PICS_TERM_ALL | PICS_TERM_WAVELET_EXPLICIT))
    return fail(c, PICS_ERR_INVALID, "apply_A_noalloc: terms %d", terms);
  if (coil_groups < 1 || coil_groups > 64)
    return fail(c, PICS_ERR_INVALID, "apply_A_noalloc: coil_groups %d outside 1..64", coil_groups);
  int need = 1;
  for (const auto& g : c->groups)
    if (g.mask_kind == PICS_MASK_LINES) need = std::max(need, std::min((int)coil_groups, g.nc_max));
  const unsigned long long bytes = need > 1 ? sizeof(float2) * (unsigned long long)c->img_total * need : 0ULL;
  if (bytes > (unsigned long long)PICS_NOALLOC_SCRATCH_BYTES)
    return fail(c, PICS_ERR_INVALID,
                "apply_A_noalloc: a coil split of %d over %lld image elements needs %llu bytes of scratch, above "
                "the %d-byte maximum (use fewer coil groups or fewer slices per context)",
                need, c->img_total, bytes, (int)PICS_NOALLOC_SCRATCH_BYTES);
  if (need > 1 && !c->scratch_dev) return fail(c, PICS_ERR_HIP, "apply_A_noalloc: scratch address not resolved");
  const bool explicit_w = (terms & PICS_TERM_WAVELET_EXPLICIT) && (terms & PICS_TERM_GAMMA);
  const int kterms = explicit_w ? (terms & (TERM_DATA | TERM_TV)) : (terms & TERM_ALL);
  {
    GroupFork fk(c);
    for (auto& g : c->groups)
      HIPCHK(c, launch_operator(c, g, CA_APPLY, kterms, c->pk, 0.0, (const float2*)x, nullptr, nullptr, nullptr,
                                (float2*)y, std::min((int)coil_groups, std::max(1, g.nc_max)), c->scratch_dev));
    HIPCHK(c, fk.join());
  }
  if (explicit_w) {
    // gam W^H W x through the wavelet kernels, in the context's workspace
    TvArgs none{};
    int rc = wavelet_analysis(c, (const float2*)x, 0, c->z, nullptr, nullptr, none);
    if (rc) return rc;
    rc = wavelet_synthesis(c, c->z, 0, c->r, nullptr, nullptr);
    if (rc) return rc;
    HIPCHK(c, launch_add_gamma(make_simple(c), make_ws(c), c->r, (const float2*)x, (float2*)y));
  }
  return PICS_OK;
}

int apply_Minv(pics_ctx* c, const void* r, void* z) {
  if (!c) return PICS_ERR_INVALID;
  if (!r || !z || r == z) return fail(c, PICS_ERR_INVALID, "apply_Minv: null or aliased buffers");
  if (c->pk != PK_CIRC && c->pk != PK_LEARNED) return fail(c, PICS_ERR_STATE, "apply_Minv: no circulant build");
  GroupFork fk(c);
  for (auto& g : c->groups) {
    HIPCHK(c, launch_row_fft(make_launch(c, g), ws_for(c, g), 0, 0, (const float2*)r, c->t));
    HIPCHK(c, launch_col_precond(make_launch(c, g), ws_for(c, g), 0, 0, 0.0, c->t, nullptr));
    HIPCHK(c, launch_row_fft(make_launch(c, g), ws_for(c, g), 1, 0, c->t, (float2*)z));
  }
  HIPCHK(c, fk.join());
  return PICS_OK;
}

int pics_fft2(pics_ctx* c, const void* in, void* out, int32_t inverse) {
  if (!c) return PICS_ERR_INVALID;
  if (!in || !out) return fail(c, PICS_ERR_INVALID, "fft2: null buffer");
  const int inv = inverse ? 1 : 0;
  GroupFork fk(c);
  for (auto& g : c->groups) {
    HIPCHK(c, launch_row_fft(make_launch(c, g), ws_for(c, g), inv, 0, (const float2*)in, c->t));
    HIPCHK(c, launch_col_fft(make_launch(c, g), ws_for(c, g), inv, c->t, (float2*)out));
  }
  HIPCHK(c, fk.join());
  return PICS_OK;
}

int pics_wavelet(pics_ctx* c, const void* in, void* out, int32_t inverse) {
  if (!c) return PICS_ERR_INVALID;
  if (!in || !out || in == out) return fail(c, PICS_ERR_INVALID, "wavelet: null or aliased buffers");
  for (int s = 0; s < c->nslices; ++s) {
    if (c->sl[s].levels == 0)
      HIPCHK(c, hipMemcpyAsync((float2*)out + c->sl[s].img, (const float2*)in + c->sl[s].img,
                               sizeof(float2) * c->sl[s].m * c->sl[s].n, hipMemcpyDeviceToDevice, c->stream));
  }
  TvArgs none{};
  if (!inverse) return wavelet_analysis(c, (const float2*)in, 0, (float2*)out, nullptr, nullptr, none);
  return wavelet_synthesis(c, (const float2*)in, 0, (float2*)out, nullptr, nullptr);
}

}  // extern "C"

// ---------------------------------------------------------------- PCG driver
namespace {

// Launch helpers read c->stream; capture swaps in the private capture stream.
struct StreamSwap {
  pics_ctx* c;
  hipStream_t saved;
  StreamSwap(pics_ctx* cc, hipStream_t s) : c(cc), saved(cc->stream) { c->stream = s; }
  ~StreamSwap() { c->stream = saved; }
};

// PCG set-up: r = b - A x0 (q already holds A x0 when q_valid), ||b||, the
// zero-iteration test, and z_0 = M^{-1} r_0 with its rho partials.
int enq_pcg_setup(pics_ctx* c, const float2* b, float2* x, double tol, int maxit, const int* maxit_dev,
                  bool q_valid) {
  const Ws w = make_ws(c);
  const int pk = c->pk;
  const bool circ = pk == PK_CIRC || pk == PK_LEARNED;
  {
    GroupFork fk(c);
    for (auto& g : c->groups) {
      if (!q_valid)
        HIPCHK(c, launch_operator(c, g, CA_APPLY, TERM_ALL, pk, tol, x, nullptr, nullptr, nullptr, c->q));
      HIPCHK(c, launch_row_update(make_launch(c, g), ws_for(c, g), RU_SETUP, pk, b, c->q, x, c->r, nullptr, nullptr,
                                  c->t, maxit, maxit_dev));
      if (circ) {
        // the set-up's stop test (zero right-hand side included) runs at
        // the start of the preconditioner's middle pass
        HIPCHK(c, launch_col_precond(make_launch(c, g), ws_for(c, g), 1, 2, tol, c->t, x));
        HIPCHK(c, launch_row_z(make_launch(c, g), ws_for(c, g), c->t, c->r, c->z));
      }
    }
    HIPCHK(c, fk.join());
  }
  if (!circ) HIPCHK(c, launch_pcg_check(c->stream, w, c->nslices, tol, 1, x));
  return PICS_OK;
}

// PCG iterations k0 .. k0 + count - 1.  Search directions alternate between
// two buffers: iteration k reads p_k from pbuf[k & 1] and writes p_{k+1} to
// pbuf[(k + 1) & 1].  Every kernel returns at entry for finished slices.
int enq_pcg_iters(pics_ctx* c, float2* x, double tol, int k0, int count) {
  const int pk = c->pk;
  const bool circ = pk == PK_CIRC || pk == PK_LEARNED;
  const float2* zsrc = circ ? c->z : c->r;
  float2* pbuf[2] = {c->p, c->pn};
  GroupFork fk(c);
  for (auto& g : c->groups) {
    for (int k = k0; k < k0 + count; ++k) {
      float2* pold = pbuf[k & 1];
      float2* pnew = pbuf[(k + 1) & 1];
      HIPCHK(c, launch_operator(c, g, CA_PCG, TERM_ALL, pk, tol, nullptr, zsrc, pold, pnew, c->q));
      HIPCHK(c, launch_row_update(make_launch(c, g), ws_for(c, g), RU_UPDATE, pk, nullptr, c->q, x, c->r, pnew,
                                  nullptr, c->t));
      if (circ) {
        HIPCHK(c, launch_col_precond(make_launch(c, g), ws_for(c, g), 1, 1, tol, c->t, nullptr));
        HIPCHK(c, launch_row_z(make_launch(c, g), ws_for(c, g), c->t, c->r, c->z));
      }
    }
  }
  HIPCHK(c, fk.join());
  return PICS_OK;
}

int pcg_status_rc(pics_ctx* c, double tol) {
  int rc = PICS_OK;
  for (int s = 0; s < c->nslices; ++s) {
    const PcgState& st = c->st_host[s];
    if (st.status < 0) rc = std::min(rc, st.status);
    else if (rc >= 0 && st.status == 0 && tol > 0.0) rc = PICS_WARN_MAXIT;
  }
  if (rc < 0) return fail(c, rc, "PCG failed: %s", pics_status_string(rc));
  return rc;
}

// One PCG solve for every slice, polled from the host: iterations are
// enqueued in chunks of 2, 4, 8, ... (at most 32) with the per-slice state
// copied back after each chunk.
int pcg_run(pics_ctx* c, const float2* b, float2* x, double tol, int maxit, const int* maxit_dev, int maxit_max,
            bool q_valid) {
  const Ws w = make_ws(c);
  int rc = enq_pcg_setup(c, b, x, tol, maxit, maxit_dev, q_valid);
  if (rc) return rc;
  int done_iters = 0;
  int chunk = std::max(1, c->poll_chunk);
  if (maxit_dev) chunk = std::max(1, maxit_max);  // iteration-locked: one poll at the end
  while (true) {
    const int todo = std::max(0, std::min(chunk, maxit_max - done_iters));
    rc = enq_pcg_iters(c, x, tol, done_iters, todo);
    if (rc) return rc;
    done_iters += todo;
    HIPCHK(c, launch_pcg_check(c->stream, w, c->nslices, tol, 0, x));
    HIPCHK(c, hipMemcpyAsync(c->st_host, c->st, sizeof(PcgState) * c->nslices, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    bool all = true;
    for (int s = 0; s < c->nslices; ++s) all = all && c->st_host[s].done;
    if (all || done_iters >= maxit_max) break;
    chunk = std::min(chunk * 2, 32);
  }
  return pcg_status_rc(c, tol);
}

// The lock schedule and history are sized by pics_create and pics_reserve;
// hot calls only check that the request fits (they never allocate).
int check_solves(pics_ctx* c, const char* who, long long solves) {
  if (solves <= c->solves_cap) return PICS_OK;
  return fail(c, PICS_ERR_INVALID, "%s: %lld solves exceed the %lld reserved for this context (pics_reserve)", who,
              solves, c->solves_cap);
}

// Split Bregman step 4: b = g_j + lam [D_x^H u_x + D_y^H u_y] + gam W^H u_w
int enq_rhs(pics_ctx* c) {
  const Ws w = make_ws(c);
  const Simple S = make_simple(c);
  if (c->any_nowavelet) HIPCHK(c, launch_rhs_nowavelet(S, w, c->g, c->ux, c->uy, c->uw, c->rhs));
  // wavelet slices: the level-0 analysis left g + lam D^H u in c->ux
  if (c->any_wavelet) return wavelet_synthesis(c, c->uw, 1, nullptr, c->ux, c->rhs);
  return PICS_OK;
}

// Split Bregman steps 6-11: TV and wavelet shrinks and Bregman updates on the
// solve's x, with the outer update fused in: q = A x = b - r for the next
// solve's set-up, and, after the last inner solve of an outer iteration
// (outer_step), steps 13-15 in the image domain, g <- g + g_1 - A_data x.
// `rec` (optional) is the solve's end record, taken by the first kernel.
// `solve` counts the solves of the reconstruction: the shrink after solve s
// reads b_x, b_y from buffer s & 1 and writes buffer (s + 1) & 1; after
// solve 0 they are still zero and not read.
int enq_shrinks(pics_ctx* c, const float2* x, bool outer_step, long long solve,
                const SolveRecord& rec = SolveRecord{}) {
  const Ws w = make_ws(c);
  const Simple S = make_simple(c);
  OuterArgs oa{outer_step ? 2 : 1, c->rhs, c->r, c->q, c->g, c->g1, rec};
  float2* bxb[2] = {c->bx, c->bx2};
  float2* byb[2] = {c->by, c->by2};
  const float2 *bxi = bxb[solve & 1], *byi = byb[solve & 1];
  float2 *bxo = bxb[(solve + 1) & 1], *byo = byb[(solve + 1) & 1];
  const int fresh = solve == 0 ? 1 : 0;
  if (c->any_nowavelet) {
    HIPCHK(c, launch_tv_shrink(S, w, 1, fresh, oa, x, bxi, byi, bxo, byo, c->ux, c->uy, c->bw, c->uw));
    oa.rec = SolveRecord{};
  }
  if (c->any_wavelet) {
    TvArgs tv{1, bxi, byi, bxo, byo, c->ux, oa, fresh};
    return wavelet_analysis(c, x, 1, nullptr, c->bw, c->uw, tv);
  }
  return PICS_OK;
}

// One outer iteration (all inner iterations) with fixed-budget PCG solves,
// each followed by a record of its per-slice iteration count and status.
// jo: index of the outer iteration in the reconstruction.
int enq_outer_iteration_budgeted(pics_ctx* c, float2* x, double tol, int n_inner, int budget, int jo) {
  for (int ji = 0; ji < n_inner; ++ji) {
    int rc = enq_rhs(c);
    if (rc) return rc;
    rc = enq_pcg_setup(c, c->rhs, x, tol, budget, nullptr, true);
    if (rc) return rc;
    rc = enq_pcg_iters(c, x, tol, 0, budget);
    if (rc) return rc;
    const SolveRecord rec{c->hist, c->hist + c->hist_cap / 2, c->solve_counter, tol, c->nslices};
    rc = enq_shrinks(c, x, ji == n_inner - 1, (long long)jo * n_inner + ji, rec);
    if (rc) return rc;
  }
  return PICS_OK;
}

// Algorithm 1, step 1 (coil images, root sum of squares, g_1, the first
// right-hand side) for every slice.
int enq_sb_init(pics_ctx* c, const float2* kspace, float2* x) {
  GroupFork fk(c);
  for (auto& g : c->groups) {
    HIPCHK(c, launch_row_fft(make_launch(c, g), ws_for(c, g), 1, 1, kspace, c->coiltmp));
    HIPCHK(c, launch_col_sb_init(make_launch(c, g), ws_for(c, g), c->coiltmp, c->g1, c->g, c->rhs, x));
  }
  HIPCHK(c, fk.join());
  return PICS_OK;
}

// The first outer iteration with fixed-budget solves: the first solve (its
// right-hand side written by the initialisation, r = b - A x0 formed by its
// set-up) carries first_budget iterations, any further inner solve budget.
int enq_first_outer_budgeted(pics_ctx* c, float2* x, double tol, int n_inner, int first_budget, int budget) {
  for (int ji = 0; ji < n_inner; ++ji) {
    int rc = ji == 0 ? PICS_OK : enq_rhs(c);
    if (rc) return rc;
    const int b = ji == 0 ? first_budget : budget;
    rc = enq_pcg_setup(c, c->rhs, x, tol, b, nullptr, ji > 0);
    if (rc) return rc;
    rc = enq_pcg_iters(c, x, tol, 0, b);
    if (rc) return rc;
    const SolveRecord rec{c->hist, c->hist + c->hist_cap / 2, c->solve_counter, tol, c->nslices};
    rc = enq_shrinks(c, x, ji == n_inner - 1, ji, rec);
    if (rc) return rc;
  }
  return PICS_OK;
}

// Capture a whole reconstruction -- the initialisation, the first outer
// iteration and the n_rep outer iterations after it -- as one graph.
int sb_graph(pics_ctx* c, const float2* kspace, float2* x, double tol, int n_inner, int first_budget, int budget,
             int n_rep) {
  const pics_ctx::GraphKey key{x, kspace, tol, budget, first_budget, c->pk, n_inner, n_rep, c->hist, c->tuning_gen};
  if (c->graph_exec && c->graph_key == key) return PICS_OK;
  if (c->graph_exec) {
    HIPCHK(c, hipGraphExecDestroy(c->graph_exec));
    c->graph_exec = nullptr;
  }
  if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  hipGraph_t graph;
  HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc;
  {
    StreamSwap sw(c, c->cap_stream);
    rc = enq_sb_init(c, kspace, x);
    if (rc == PICS_OK) rc = enq_first_outer_budgeted(c, x, tol, n_inner, first_budget, budget);
    for (int k = 0; k < n_rep && rc == PICS_OK; ++k)
      rc = enq_outer_iteration_budgeted(c, x, tol, n_inner, budget, 1 + k);
  }
  const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
  if (rc) {
    if (e == hipSuccess) (void)hipGraphDestroy(graph);
    return rc;
  }
  HIPCHK(c, e);
  const hipError_t ei = hipGraphInstantiate(&c->graph_exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIPCHK(c, ei);
  c->graph_key = key;
  return PICS_OK;
}

}  // namespace

extern "C" {

int pcg_solve(pics_ctx* c, const void* b, void* x, double tol, int32_t maxit, const int32_t* maxit_per_slice,
              int32_t* iters_host, double* relres_host, int32_t* status_host) {
  if (!c) return PICS_ERR_INVALID;
  if (!b || !x || b == x) return fail(c, PICS_ERR_INVALID, "pcg_solve: null or aliased buffers");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(c, PICS_ERR_INVALID, "pcg_solve: tol");
  if (maxit < 0) return fail(c, PICS_ERR_INVALID, "pcg_solve: maxit");
  int maxit_max = maxit;
  const int* mdev = nullptr;
  if (maxit_per_slice) {
    maxit_max = 0;
    for (int s = 0; s < c->nslices; ++s) {
      if (maxit_per_slice[s] < 0) return fail(c, PICS_ERR_INVALID, "pcg_solve: maxit_per_slice");
      maxit_max = std::max(maxit_max, (int)maxit_per_slice[s]);
    }
    HIPCHK(c, hipMemcpyAsync(c->lock_dev, maxit_per_slice, sizeof(int) * c->nslices, hipMemcpyHostToDevice,
                             c->stream));
    mdev = c->lock_dev;
  }
  const int rc = pcg_run(c, (const float2*)b, (float2*)x, tol, maxit, mdev, maxit_max, false);
  for (int s = 0; s < c->nslices; ++s) {
    if (iters_host) iters_host[s] = c->st_host[s].iters;
    if (relres_host) relres_host[s] = c->st_host[s].relres;
    if (status_host) status_host[s] = c->st_host[s].status;
  }
  return rc;
}

int split_bregman_recon(pics_ctx* c, const void* kspace, int32_t n_outer, int32_t n_inner, double tol,
                        int32_t maxit, const int32_t* lock_iters, void* x_out, int32_t* pcg_iters) {
  if (!c) return PICS_ERR_INVALID;
  if (!kspace || !x_out) return fail(c, PICS_ERR_INVALID, "split_bregman_recon: null buffer");
  if (n_outer < 0 || n_inner < 1 || maxit < 0 || !(tol >= 0.0))
    return fail(c, PICS_ERR_INVALID, "split_bregman_recon: iteration parameters");
  for (int s = 0; s < c->nslices; ++s)
    if (!(c->desc[s].lambda > 0.0) || !(c->desc[s].gamma > 0.0))
      return fail(c, PICS_ERR_INVALID, "split_bregman_recon: lambda and gamma must be > 0 (shrink thresholds)");
  const long long nsolve = (long long)n_outer * n_inner;
  if (nsolve > 0) {
    const int rc = check_solves(c, "split_bregman_recon", nsolve);
    if (rc) return rc;
  }
  if (lock_iters) {
    HIPCHK(c, hipMemcpyAsync(c->lock_dev, lock_iters, sizeof(int) * nsolve * c->nslices, hipMemcpyHostToDevice,
                             c->stream));
  }
  float2* x = (float2*)x_out;
  const bool use_graph = !lock_iters && c->graph_budget > 0 && n_outer > 1 && tol > 0.0;
  if (use_graph) {
    // the whole reconstruction from one graph: fixed-budget solves whose
    // kernels exit at entry once a slice has converged, and a device record
    // of every solve's count and status
    const int budget = std::min(c->graph_budget, maxit);
    const int first_budget = std::min(c->graph_first_budget, maxit);
    int rc = sb_graph(c, (const float2*)kspace, x, tol, n_inner, first_budget, budget, n_outer - 1);
    if (rc) return rc;
    HIPCHK(c, launch_set_int(c->stream, c->solve_counter, 0));
    HIPCHK(c, hipGraphLaunch(c->graph_exec, c->stream));
    const long long rows = nsolve * c->nslices;
    c->hist_host.resize(2 * rows);
    HIPCHK(c, hipMemcpyAsync(c->hist_host.data(), c->hist, sizeof(int) * rows, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->hist_host.data() + rows, c->hist + c->hist_cap / 2, sizeof(int) * rows,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    bool over_first = false, over = false;
    int mx = 0;
    for (long long r = 0; r < rows; ++r) {
      const int st = c->hist_host[rows + r];
      if (st < 0) return fail(c, st, "PCG failed inside the reconstruction graph: %s", pics_status_string(st));
      if (st == 0) (r < c->nslices ? over_first : over) = true;
      if (r >= c->nslices) mx = std::max(mx, c->hist_host[r]);
    }
    if (!over_first && !over) {
      if (pcg_iters)
        for (long long r = 0; r < rows; ++r) pcg_iters[r] = c->hist_host[r];
      return PICS_OK;
    }
    // a solve needed more than its budget: redo the reconstruction
    // host-polled (results never depend on the budgets) and raise the budget
    if (over_first) c->graph_first_budget = std::min(256, 2 * c->graph_first_budget);
    if (over) c->graph_budget = std::min(64, std::max(c->graph_budget < 2 ? 2 : c->graph_budget * 2, mx + 1));
    c->graph_fallbacks++;
  }
  // host-polled: Algorithm 1, step 1, then every solve polled to convergence
  int rc = enq_sb_init(c, (const float2*)kspace, x);
  if (rc) return rc;
  // b_x = b_y = b_w = 0 and d = 0 at the start: the first right-hand side
  // is g (written by the initialisation) and the first shrinks read no
  // Bregman variables
  bool q_valid = false;
  int rc_all = PICS_OK;
  for (int jo = 0; jo < n_outer; ++jo) {
    for (int ji = 0; ji < n_inner; ++ji) {
      const long long solve = (long long)jo * n_inner + ji;
      rc = solve == 0 ? PICS_OK : enq_rhs(c);
      if (rc) return rc;
      if (lock_iters) {
        int mx = 0;
        for (int s = 0; s < c->nslices; ++s) mx = std::max(mx, (int)lock_iters[solve * c->nslices + s]);
        rc = pcg_run(c, c->rhs, x, 0.0, 0, c->lock_dev + solve * c->nslices, mx, q_valid);
      } else {
        rc = pcg_run(c, c->rhs, x, tol, maxit, nullptr, maxit, q_valid);
      }
      if (rc < 0) return rc;
      if (rc > 0) rc_all = rc;
      if (pcg_iters)
        for (int s = 0; s < c->nslices; ++s) pcg_iters[solve * c->nslices + s] = c->st_host[s].iters;
      rc = enq_shrinks(c, x, ji == n_inner - 1, solve);
      if (rc) return rc;
      q_valid = true;  // the shrinks left A x = b - r in q
    }
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return rc_all;
}

}  // extern "C"

extern "C" {

int pics_coil_compress(pics_ctx* c, const void* kspace, int32_t nvirt, void* kspace_out, void* sens_out,
                       double* eig_out) {
  if (!c) return PICS_ERR_INVALID;
  if (!kspace || !kspace_out || !sens_out) return fail(c, PICS_ERR_INVALID, "coil_compress: null buffer");
  for (const SliceDev& sd : c->sl) {
    if (sd.nc > 32) return fail(c, PICS_ERR_UNSUPPORTED, "coil_compress: at most 32 coils per slice");
    if (nvirt < 1 || nvirt > sd.nc) return fail(c, PICS_ERR_INVALID, "coil_compress: nvirt %d out of range", nvirt);
  }
  const Ws w = make_ws(c);
  HIPCHK(c, launch_coil_compress(make_simple(c), w, (const float2*)kspace, c->sens, nvirt, (double2*)c->coiltmp,
                                 (float2*)kspace_out, (float2*)sens_out));
  if (eig_out) {
    std::vector<double> slots((size_t)c->nslices * kSlots * kPartMax);
    HIPCHK(c, hipMemcpyAsync(slots.data(), c->part, sizeof(double) * slots.size(), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    long long o = 0;
    for (int s = 0; s < c->nslices; ++s)
      for (int k = 0; k < c->sl[s].nc; ++k) eig_out[o++] = slots[((size_t)s * kSlots + P_AUX) * kPartMax + k];
  }
  return PICS_OK;
}

}  // extern "C"

// =================================================================== learned
namespace {
const int kLayerSpec[kNetLayers][3] = {{6, 32, 1}, {32, 32, 1}, {32, 32, 2}, {32, 32, 4}, {32, 32, 8}, {32, 16, 1}};
}

struct pics_net {
  hipStream_t stream = nullptr;
  int bmax = 0;
  void* block = nullptr;
  NetLayout L{};
  float *theta, *grad, *m, *v;
  uint16_t* act[kNetLayers + 1];
  uint16_t* gbuf[2];
  float *o, *go, *part;
  double *loss_part, *zsum;
  double* loss_host = nullptr;  // pinned
  int t = 0;
  bool prepped = false;
  std::string err;
};

namespace {
int nfail(pics_net* n, int code, const char* msg) {
  if (n) n->err = msg;
  return code;
}
#define NETCHK(net, expr)                                              \
  do {                                                                 \
    hipError_t e_ = (expr);                                            \
    if (e_ != hipSuccess) return nfail(net, PICS_ERR_HIP, hipGetErrorString(e_)); \
  } while (0)

int net_prep(pics_net* n) {
  if (!n->prepped) {
    NETCHK(n, launch_net_prep(n->stream, n->theta, n->L));
    n->prepped = true;
  }
  return PICS_OK;
}

int net_forward(pics_net* n, int batch, const int* index, const float* feat) {
  int rc = net_prep(n);
  if (rc) return rc;
  NETCHK(n, launch_net_input(n->stream, feat, index, batch, n->act[0]));
  for (int l = 0; l < kNetLayers; ++l) {
    const NetLayer& ly = n->L.layer[l];
    NETCHK(n, launch_conv_fwd(n->stream, ly.cinp, ly.cout, n->act[l], ly.wf, n->theta + ly.woff + ly.cout * ly.cin * 9,
                              ly.dil, batch, n->act[l + 1]));
  }
  return PICS_OK;
}
}  // namespace

extern "C" {

int64_t pics_net_param_count(void) {
  long long c = 0;
  for (int l = 0; l < kNetLayers; ++l) c += (long long)kLayerSpec[l][1] * kLayerSpec[l][0] * 9 + kLayerSpec[l][1];
  return c + 17;
}

int pics_net_create(pics_net** out, int32_t batch_max, void* stream) {
  if (!out || batch_max < 1 || batch_max > 4096) return PICS_ERR_INVALID;
  *out = nullptr;
  pics_net* n = new pics_net();
  n->stream = (hipStream_t)stream;
  n->bmax = batch_max;
  long long off = 0;
  for (int l = 0; l < kNetLayers; ++l) {
    NetLayer& ly = n->L.layer[l];
    ly.cin = kLayerSpec[l][0];
    ly.cout = kLayerSpec[l][1];
    ly.dil = kLayerSpec[l][2];
    ly.cinp = ly.cin <= 16 ? 16 : 32;
    ly.woff = off;
    off += (long long)ly.cout * ly.cin * 9 + ly.cout;
  }
  n->L.final_off = off;
  n->L.count = off + 17;
  const long long P = n->L.count;
  const long long cells = (long long)kNetGrid * kNetGrid;
  std::vector<std::pair<void**, size_t>> plan;
  auto add = [&](void** p, size_t bytes) { plan.push_back({p, (bytes + 255) / 256 * 256}); };
  add((void**)&n->theta, sizeof(float) * P);
  add((void**)&n->grad, sizeof(float) * P);
  add((void**)&n->m, sizeof(float) * P);
  add((void**)&n->v, sizeof(float) * P);
  for (int l = 0; l < kNetLayers; ++l) {
    NetLayer& ly = n->L.layer[l];
    add((void**)&ly.wf, sizeof(uint16_t) * ly.cout * 9 * ly.cinp);
    add((void**)&ly.wb, sizeof(uint16_t) * ly.cout * 9 * ly.cinp);
  }
  add((void**)&n->act[0], sizeof(uint16_t) * batch_max * cells * 16);
  for (int l = 0; l < kNetLayers; ++l)
    add((void**)&n->act[l + 1], sizeof(uint16_t) * batch_max * cells * n->L.layer[l].cout);
  for (int i = 0; i < 2; ++i) add((void**)&n->gbuf[i], sizeof(uint16_t) * batch_max * cells * 32);
  add((void**)&n->o, sizeof(float) * batch_max * cells);
  add((void**)&n->go, sizeof(float) * batch_max * cells);
  add((void**)&n->part, sizeof(float) * batch_max * kNetGrid * (32 * 32 * 9 + 32));
  add((void**)&n->loss_part, sizeof(double) * batch_max * kNetGrid);
  add((void**)&n->zsum, sizeof(double) * batch_max);
  size_t total = 0;
  for (auto& pr : plan) total += pr.second;
  if (hipMalloc(&n->block, total) != hipSuccess) {
    delete n;
    return PICS_ERR_HIP;
  }
  char* base = (char*)n->block;
  for (auto& pr : plan) {
    *pr.first = base;
    base += pr.second;
  }
  if (hipHostMalloc((void**)&n->loss_host, sizeof(double) * batch_max * kNetGrid, hipHostMallocDefault) != hipSuccess ||
      hipMemset(n->block, 0, total) != hipSuccess) {
    if (n->loss_host) (void)hipHostFree(n->loss_host);
    (void)hipFree(n->block);
    delete n;
    return PICS_ERR_HIP;
  }
  *out = n;
  return PICS_OK;
}

int pics_net_destroy(pics_net* n) {
  if (!n) return PICS_ERR_INVALID;
  (void)hipStreamSynchronize(n->stream);
  if (n->loss_host) (void)hipHostFree(n->loss_host);
  if (n->block) (void)hipFree(n->block);
  delete n;
  return PICS_OK;
}

int pics_net_set_params(pics_net* n, const float* params) {
  if (!n || !params) return PICS_ERR_INVALID;
  NETCHK(n, hipMemcpyAsync(n->theta, params, sizeof(float) * n->L.count, hipMemcpyHostToDevice, n->stream));
  NETCHK(n, hipMemsetAsync(n->m, 0, sizeof(float) * n->L.count, n->stream));
  NETCHK(n, hipMemsetAsync(n->v, 0, sizeof(float) * n->L.count, n->stream));
  NETCHK(n, hipStreamSynchronize(n->stream));
  n->t = 0;
  n->prepped = false;
  return PICS_OK;
}

int pics_net_get_params(pics_net* n, float* params) {
  if (!n || !params) return PICS_ERR_INVALID;
  NETCHK(n, hipMemcpyAsync(params, n->theta, sizeof(float) * n->L.count, hipMemcpyDeviceToHost, n->stream));
  NETCHK(n, hipStreamSynchronize(n->stream));
  return PICS_OK;
}

int pics_net_get_grad(pics_net* n, float* g) {
  if (!n || !g) return PICS_ERR_INVALID;
  NETCHK(n, hipMemcpyAsync(g, n->grad, sizeof(float) * n->L.count, hipMemcpyDeviceToHost, n->stream));
  NETCHK(n, hipStreamSynchronize(n->stream));
  return PICS_OK;
}

int pics_net_forward(pics_net* n, int32_t batch, const int32_t* index, const float* feat, float* o) {
  if (!n || !feat || !o || batch < 1 || batch > n->bmax) return PICS_ERR_INVALID;
  int rc = net_forward(n, batch, index, feat);
  if (rc) return rc;
  NETCHK(n, launch_net_head(n->stream, n->act[kNetLayers], n->theta, (int)n->L.final_off, index, batch, nullptr,
                            nullptr, nullptr, nullptr, nullptr, o, nullptr, n->loss_part));
  return PICS_OK;
}

int pics_net_loss_grad(pics_net* n, int32_t batch, const int32_t* index, const float* feat, const float* k,
                       const float* G, const float* H, const float* Z, double* loss_host) {
  if (!n || !feat || !k || !G || !H || !Z || batch < 1 || batch > n->bmax) return PICS_ERR_INVALID;
  if (!index) return nfail(n, PICS_ERR_INVALID, "loss_grad needs a device index array");
  int rc = net_forward(n, batch, index, feat);
  if (rc) return rc;
  // zsum[b] = sum_j Z_j of slice index[b]
  NETCHK(n, launch_plane_sums_indexed(n->stream, Z, index, batch, n->zsum));
  NETCHK(n, launch_net_head(n->stream, n->act[kNetLayers], n->theta, (int)n->L.final_off, index, batch, k, G, H, Z,
                            n->zsum, n->o, n->go, n->loss_part));
  // backward
  const long long rows = (long long)batch * kNetGrid;
  NETCHK(n, launch_net_head_bwd(n->stream, n->act[kNetLayers], n->theta, (int)n->L.final_off, n->go, batch, n->gbuf[0],
                                n->part));
  NETCHK(n, launch_reduce_rows(n->stream, n->part, (int)rows, 17, n->grad + n->L.final_off));
  int cur = 0;
  for (int l = kNetLayers - 1; l >= 0; --l) {
    const NetLayer& ly = n->L.layer[l];
    const int count = ly.cout * ly.cin * 9 + ly.cout;
    NETCHK(n, launch_conv_bwd_w(n->stream, ly.cinp, ly.cin, ly.cout, n->act[l], n->gbuf[cur], ly.dil, batch, n->part));
    NETCHK(n, launch_reduce_rows(n->stream, n->part, (int)(rows / kWgRows), count, n->grad + ly.woff));
    if (l > 0) {
      NETCHK(n, launch_conv_bwd_data(n->stream, ly.cinp, ly.cout, n->gbuf[cur], ly.wb, n->act[l], ly.dil, batch,
                                     n->gbuf[1 - cur]));
      cur = 1 - cur;
    }
  }
  NETCHK(n, hipMemcpyAsync(n->loss_host, n->loss_part, sizeof(double) * rows, hipMemcpyDeviceToHost, n->stream));
  NETCHK(n, hipStreamSynchronize(n->stream));
  if (loss_host) {
    double acc = 0.0;
    for (long long r = 0; r < rows; ++r) acc += n->loss_host[r];
    *loss_host = acc / batch;
  }
  return PICS_OK;
}

int pics_net_adam_step(pics_net* n, float lr) {
  if (!n || !(lr > 0.f)) return PICS_ERR_INVALID;
  n->t++;
  NETCHK(n, launch_adam(n->stream, n->theta, n->grad, n->m, n->v, (int)n->L.count, lr, n->t));
  n->prepped = false;
  return PICS_OK;
}

int pics_features(pics_ctx* c, const float* khat, float* features) {
  if (!c || !khat || !features) return PICS_ERR_INVALID;
  for (const SliceDev& sd : c->sl)
    if (sd.m % kNetGrid || sd.n % kNetGrid) return fail(c, PICS_ERR_UNSUPPORTED, "features need m, n multiples of 64");
  {
    GroupFork fk(c);
    for (auto& g : c->groups) {
      HIPCHK(c, launch_row_fft(make_launch(c, g), ws_for(c, g), 0, 2, c->sens, c->coiltmp));
      HIPCHK(c, launch_col_coil_energy(make_launch(c, g), ws_for(c, g), c->coiltmp, c->ftmp));
    }
    HIPCHK(c, fk.join());
  }
  HIPCHK(c, launch_features(c->stream, make_ws(c), c->nslices, c->ftmp, khat, features));
  return PICS_OK;
}

int pics_probe_stats(pics_ctx* c, const void* probes, int32_t nprobes, float* G, float* H, float* Z) {
  if (!c || !probes || nprobes < 1 || !G || !H || !Z) return PICS_ERR_INVALID;
  const float2* pr = (const float2*)probes;
  for (int p = 0; p < nprobes; ++p) {
    const float2* z = pr + (long long)p * c->img_total;
    int rc = apply_A(c, z, c->w1, PICS_TERM_ALL);
    if (rc) return rc;
    rc = pics_fft2(c, c->w1, c->w1, 0);
    if (rc) return rc;
    rc = pics_fft2(c, z, c->w2, 0);
    if (rc) return rc;
    HIPCHK(c, launch_probe_accum(make_simple(c), make_ws(c), c->w1, c->w2, G, H, Z, 1.0f / nprobes, p == 0));
  }
  return PICS_OK;
}

int pics_net_correction(pics_net* n, pics_ctx* c, const float* features, float* corr) {
  if (!n || !c || !features || !corr) return PICS_ERR_INVALID;
  HIPCHK(c, hipStreamSynchronize(c->stream));  // features come from the context's stream
  const long long cells = (long long)kNetGrid * kNetGrid;
  for (int s0 = 0; s0 < c->nslices; s0 += n->bmax) {
    const int b = std::min(n->bmax, c->nslices - s0);
    int rc = pics_net_forward(n, b, nullptr, features + (long long)s0 * kNetFeat * cells, n->o);
    if (rc) return fail(c, rc, n->err.c_str());
    HIPCHK(c, launch_net_upsample(n->stream, make_ws(c), n->o, s0, b, c->max_pixels, corr));
  }
  HIPCHK(c, hipStreamSynchronize(n->stream));
  return PICS_OK;
}

}  // extern "C"

// ================================================================= autotuner
// Per group of equal-size slices, time the fused operator for each launch
// shape: the default column tiles with each coil split (1, 2, 3, 4, 6, 8, 12
// workgroups per tile), and the two alternative tile widths of the length
// without a split; keep the fastest (HIP events).  Results are cached per
// (GPU arch, CU count, m, n, largest coil count, slices in the group) in a
// text file ($PICS_TUNE_CACHE, default ~/.cache/pics_autotune.txt) as
// tile x 100 + split.
namespace {

std::atomic<long> tune_tmp_counter{0};
std::mutex tune_mutex;  // one autotuning pass per process at a time (shared cache file)

std::string tune_cache_path() {
  const char* p = getenv("PICS_TUNE_CACHE");
  if (p && *p) return p;
  const char* h = getenv("HOME");
  return std::string(h ? h : "/tmp") + "/.cache/pics_autotune.txt";
}

std::string device_tag() {
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  char buf[128];
  snprintf(buf, sizeof buf, "%s/%d", prop.gcnArchName, prop.multiProcessorCount);
  for (char* q = buf; *q; ++q)
    if (*q == ' ' || *q == ':') *q = '_';
  return buf;
}

// v2: the split applies to the group's slice with the most coils, the
// others take workgroups in proportion (entries of the uniform split are
// not reused)
std::string group_key(const pics_ctx::Group& g) {
  char buf[160];
  snprintf(buf, sizeof buf, "v2 %s m%d n%d nc%d b%d", device_tag().c_str(), g.m, g.n, g.nc_max, (int)g.idx.size());
  return buf;
}

std::map<std::string, int> read_tune_cache() {
  std::map<std::string, int> out;
  FILE* f = fopen(tune_cache_path().c_str(), "r");
  if (!f) return out;
  char line[256];
  while (fgets(line, sizeof line, f)) {
    std::string l(line);
    const size_t eq = l.rfind('=');
    if (eq == std::string::npos) continue;
    out[l.substr(0, eq)] = atoi(l.c_str() + eq + 1);
  }
  fclose(f);
  return out;
}

void write_tune_cache(const std::map<std::string, int>& m) {
  const std::string path = tune_cache_path();
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos) {
    // create the directory (and its parents) without a shell
    const std::string dir = path.substr(0, slash);
    for (size_t i = 1; i <= dir.size(); ++i)
      if (i == dir.size() || dir[i] == '/') mkdir(dir.substr(0, i).c_str(), 0755);
  }
  // written to a private file and renamed over the cache, so that a reader
  // (another context or process) sees either the old or the new file whole
  const std::string tmp = path + ".tmp." + std::to_string((long)getpid()) + "." +
                          std::to_string(tune_tmp_counter.fetch_add(1));
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  for (auto& kv : m) fprintf(f, "%s=%d\n", kv.first.c_str(), kv.second);
  if (fclose(f) != 0 || rename(tmp.c_str(), path.c_str()) != 0) remove(tmp.c_str());
}

int ensure_dpart(pics_ctx* c, int groups) {
  if (groups <= c->dpart_groups) return PICS_OK;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->dpart) HIPCHK(c, hipFree(c->dpart));
  c->dpart = nullptr;
  HIPCHK(c, hipMalloc((void**)&c->dpart, sizeof(float2) * c->img_total * groups));
  c->dpart_groups = groups;
  ++c->tuning_gen;
  return PICS_OK;
}

}  // namespace

extern "C" {

int pics_autotune(pics_ctx* c, int32_t flags) {
  if (!c) return PICS_ERR_INVALID;
  std::lock_guard<std::mutex> lock(tune_mutex);
  std::map<std::string, int> cache = (flags & PICS_TUNE_FORCE) ? std::map<std::string, int>() : read_tune_cache();
  bool changed = false;
  struct Events {  // destroyed on every return path
    hipEvent_t e[2] = {nullptr, nullptr};
    ~Events() {
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev;
  HIPCHK(c, hipEventCreate(&ev.e[0]));
  HIPCHK(c, hipEventCreate(&ev.e[1]));
  hipEvent_t e0 = ev.e[0], e1 = ev.e[1];
  HIPCHK(c, launch_fill(c->stream, c->p, c->img_total, make_float2(1.f, 0.5f)));
  for (auto& g : c->groups) {
    if (g.mask_kind == PICS_MASK_2D) continue;  // the 2D path has no coil split
    const std::string key = group_key(g);
    const int tdef = col_tile(g.m);
    auto hit = cache.find(key);
    if (hit != cache.end()) {
      // cached value: tile x 100 + coil split (a bare split: the default tiles)
      const int v = hit->second, tile = v >= 100 ? v / 100 : tdef, G = v >= 100 ? v % 100 : v;
      if (G >= 1 && G <= g.nc_max && apply_tile_ok(g.m, g.n, tile) && (G == 1 || tile == tdef)) {
        int rc = ensure_dpart(c, G);
        if (!rc) rc = set_group_tile(c, g, tile);
        if (rc) return rc;
        g.coil_groups = G;
        continue;
      }
    }
    // candidates: the default tiles with each coil split, then the two
    // alternative tile widths without a split
    std::vector<std::pair<int, int>> cands;
    for (int G : {1, 2, 3, 4, 6, 8, 12})
      if (G <= g.nc_max) cands.push_back({tdef, G});
    for (int k = 0; k < 2; ++k)
      if (apply_tile_ok(g.m, g.n, apply_tile_alt(g.m, k))) cands.push_back({apply_tile_alt(g.m, k), 1});
    float best_ms = 1e30f;
    std::pair<int, int> best{tdef, 1};
    for (auto cand : cands) {
      const int tile = cand.first, G = cand.second;
      int rc = ensure_dpart(c, G);
      if (rc) return rc;
      auto run = [&]() {
        return launch_col_apply(make_launch(c, g), ws_for(c, g), CA_APPLY, TERM_ALL, c->pk, 0.0, c->p, nullptr,
                                nullptr, nullptr, c->q, G, c->dpart, c->img_total, tile, g.nc_max);
      };
      for (int k = 0; k < 2; ++k) HIPCHK(c, run());
      HIPCHK(c, hipEventRecord(e0, c->stream));
      const int reps = 10;
      for (int k = 0; k < reps; ++k) HIPCHK(c, run());
      HIPCHK(c, hipEventRecord(e1, c->stream));
      HIPCHK(c, hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
      ms /= reps;
      if (ms < best_ms * 0.97f) {  // a later candidate must win by 3% to be taken
        best_ms = ms;
        best = cand;
      }
    }
    int rc = set_group_tile(c, g, best.first);
    if (rc) return rc;
    g.coil_groups = best.second;
    cache[key] = best.first * 100 + best.second;
    changed = true;
  }
  ++c->tuning_gen;
  if (changed && !(flags & PICS_TUNE_NO_WRITE)) write_tune_cache(cache);
  return PICS_OK;
}

int pics_get_tuning(const pics_ctx* c, int32_t* coil_groups, int32_t max_groups) {
  if (!c || !coil_groups) return PICS_ERR_INVALID;
  for (int i = 0; i < (int)c->groups.size() && i < max_groups; ++i) coil_groups[i] = c->groups[i].coil_groups;
  return (int)c->groups.size();
}

int pics_get_tuning_tiles(const pics_ctx* c, int32_t* tiles, int32_t max_groups) {
  if (!c || !tiles) return PICS_ERR_INVALID;
  for (int i = 0; i < (int)c->groups.size() && i < max_groups; ++i) {
    const auto& g = c->groups[i];
    tiles[i] = g.mask_kind == PICS_MASK_LINES ? (g.tile ? g.tile : col_tile(g.m)) : 0;
  }
  return (int)c->groups.size();
}

}  // extern "C"
