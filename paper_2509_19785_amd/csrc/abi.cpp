// Host side of the C ABI: argument validation, ownership of device memory,
// dispatch of the evaluation stages onto the caller's stream, stage timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "tsnet_internal.h"

struct tsnet_ctx_s {
  tsnet::Ctx c;
};
struct tsnet_P_s {
  tsnet::Problem p;
};

namespace tsnet {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

static const char* kStageNames[ST_COUNT] = {"bbox_plan", "bin_sort", "spread", "fft_conv",
                                             "gather", "z_reduce", "attract_assemble", "step",
                                             "cost", "direct_f64", "build_P", "pmds",
                                             "np", "stress", "quadtree", "far_points"};

template <typename T>
static int dmalloc(T** p, size_t count, const char* what) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(e == hipErrorOutOfMemory ? TSNET_ENOMEM : TSNET_EHIP,
                std::string("hipMalloc(") + what + "): " + hipGetErrorString(e));
  }
  return TSNET_OK;
}

template <typename T>
static void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// ---------------------------------------------------------------- timing
struct StageScope {
  Ctx& c;
  int st;
  hipStream_t s;
  hipEvent_t a = nullptr;
  StageScope(Ctx& c_, int st_, hipStream_t s_) : c(c_), st(st_), s(s_) {
    if (!(c.timing & (1u << st))) return;
    a = take_event();
    if (a) (void)hipEventRecord(a, s);
  }
  hipEvent_t take_event() {
    if (!c.ev_free.empty()) {
      hipEvent_t e = c.ev_free.back();
      c.ev_free.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  ~StageScope() {
    if (!a) return;
    hipEvent_t b = take_event();
    if (!b) {
      c.ev_free.push_back(a);
      return;
    }
    (void)hipEventRecord(b, s);
    c.pending.push_back({st, a, b});
  }
};

static int collect_times(Ctx& c) {
  for (auto& p : c.pending) {
    TSNET_HIP(hipEventSynchronize(p.b));
    float ms = 0.f;
    TSNET_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    c.stage_ms[p.stage] += ms;
    c.stage_calls[p.stage] += 1;
    c.ev_free.push_back(p.a);
    c.ev_free.push_back(p.b);
  }
  c.pending.clear();
  return TSNET_OK;
}

// ---------------------------------------------------------------- problems
static void free_pools(Problem& P) {
  dfree(P.charges);
  dfree(P.qspec);
  dfree(P.qspec_t);
  dfree(P.kspec);
  dfree(P.kspec_t);
  dfree(P.ospec);
  dfree(P.ospec_t);
  dfree(P.pot);
  for (int k = 0; k < POOL_KINDS; ++k) P.pool_cap[k] = 0;
}

// Pools of the grid buffers with `cap[k]` elements of each kind.
static int alloc_pools(Problem& P, const size_t* cap) {
  int rc;
  if ((rc = dmalloc(&P.charges, cap[POOL_C], "charges")) ||
      (rc = dmalloc(&P.qspec, cap[POOL_Q], "qspec")) ||
      (rc = dmalloc(&P.qspec_t, cap[POOL_Q], "qspec")) ||
      (rc = dmalloc(&P.kspec, cap[POOL_K], "kspec")) ||
      (rc = dmalloc(&P.kspec_t, cap[POOL_K], "kspec")) ||
      (rc = dmalloc(&P.ospec, cap[POOL_O], "ospec")) ||
      (rc = dmalloc(&P.ospec_t, cap[POOL_O], "ospec")) ||
      (rc = dmalloc(&P.pot, cap[POOL_P], "pot"))) {
    free_pools(P);
    return rc;
  }
  for (int k = 0; k < POOL_KINDS; ++k) P.pool_cap[k] = cap[k];
  return TSNET_OK;
}

static void free_grid(Problem& P) {
  dfree(P.box_off);
  dfree(P.trim_hist);
  free_pools(P);
  if (P.need_host) (void)hipHostFree(P.need_host);
  P.need_host = nullptr;
  P.need_dev = nullptr;
  P.cap = 0;
}

static void free_problem(Problem& P) {
  if (P.ctx) {
    --P.ctx->live_problems;
    P.ctx = nullptr;
  }
  free_grid(P);
  free_quadtree(P);
  dfree(P.ginfo);
  dfree(P.goff_d);
  dfree(P.vgraph);
  dfree(P.chunk_graph);
  dfree(P.chunk_start);
  dfree(P.chunk_end);
  dfree(P.rowptr);
  dfree(P.col);
  dfree(P.val);
  dfree(P.tile_rows);
  dfree(P.tile_wlo);
  dfree(P.tile_boff);
  dfree(P.tile_graph);
  dfree(P.tile_order);
  dfree(P.tile_bstart);
  dfree(P.tile_ent);
  P.tile_T = P.tile_R = 0;
  P.tile_NB = 0;
  dfree(P.beta);
  dfree(P.rstatus);
  dfree(P.cond_len);
  dfree(P.cond_nbr);
  dfree(P.cond_dist);
  dfree(P.desc);
  dfree(P.bbox_part);
  dfree(P.btotal);
  dfree(P.keys);
  dfree(P.keys_tmp);
  dfree(P.perm_tmp);
  dfree(P.perm_tmp2);
  dfree(P.skeys);
  dfree(P.perm);
  dfree(P.xs);
  dfree(P.bin_hist);
  dfree(P.bin_rtot);
  dfree(P.row_order);
  dfree(P.head_box);
  dfree(P.tail_box);
  dfree(P.head_val);
  dfree(P.tail_val);
  dfree(P.rep_ent);
  dfree(P.zi);
  dfree(P.lnv);
  dfree(P.slot_z);
  dfree(P.slot_ln);
  dfree(P.zpart);
  dfree(P.zg);
  dfree(P.cost_part);
  dfree(P.direct_part);
}

static int check_offsets(int n, const int32_t* goff_host, int G, std::vector<int>& out) {
  if (G < 1) return fail(TSNET_EINVAL, "num_graphs must be >= 1");
  out.assign(G + 1, 0);
  if (!goff_host) {
    if (G != 1) return fail(TSNET_EINVAL, "graph_offsets_host is NULL but num_graphs != 1");
    out[1] = n;
    return TSNET_OK;
  }
  for (int g = 0; g <= G; ++g) out[g] = goff_host[g];
  if (out[0] != 0 || out[G] != n)
    return fail(TSNET_EINVAL, "graph_offsets must start at 0 and end at n");
  for (int g = 0; g < G; ++g)
    if (out[g + 1] <= out[g]) return fail(TSNET_EINVAL, "every graph needs at least one vertex");
  return TSNET_OK;
}

// Graph tables, chunk tables and the per-vertex workspace shared by every problem.
static int init_problem(Ctx& c, Problem& P, int n, const int32_t* goff_host, int G) {
  P.ctx = &c;
  ++c.live_problems;
  if (n < 1) return fail(TSNET_EINVAL, "n must be >= 1");
  int rc = check_offsets(n, goff_host, G, P.goff);
  if (rc) return rc;
  P.n = n;
  P.G = G;
  std::vector<int> cg, cs, ce;
  P.ginfo_h.resize(G);
  for (int g = 0; g < G; ++g) {
    GraphInfo gi{};
    gi.vstart = P.goff[g];
    gi.n = P.goff[g + 1] - P.goff[g];
    gi.chunk_begin = (int)cg.size();
    for (int s = P.goff[g]; s < P.goff[g + 1]; s += kChunk) {
      cg.push_back(g);
      cs.push_back(s);
      ce.push_back(std::min(s + kChunk, P.goff[g + 1]));
    }
    gi.chunk_end = (int)cg.size();
    gi.inv_n = (float)(1.0 / gi.n);
    gi.inv_n2 = (float)(1.0 / ((double)gi.n * gi.n));
    gi.lr = (float)std::max(200.0, gi.n / 12.0);
    P.ginfo_h[g] = gi;
  }
  P.num_chunks = (int)cg.size();
  const int nc = P.num_chunks;
  const size_t tiles = ((size_t)n + kBinTileH - 1) / kBinTileH;
  // sorted points per wave of the spread: kSpreadRange, halved (down to 64)
  // while the problem has fewer than 2048 ranges (8 waves per CU), so the
  // spread of all but the largest problems still keeps the chip busy
  int sr = kSpreadRange;
  while (sr > 64 && ((size_t)n + sr - 1) / sr < 2048) sr >>= 1;
  P.spread_range = sr;
  const size_t ranges = ((size_t)n + sr - 1) / sr;
  if ((rc = dmalloc(&P.ginfo, G, "ginfo")) || (rc = dmalloc(&P.goff_d, G + 1, "goff")) ||
      (rc = dmalloc(&P.chunk_graph, nc, "chunks")) || (rc = dmalloc(&P.chunk_start, nc, "chunks")) ||
      (rc = dmalloc(&P.chunk_end, nc, "chunks")) || (rc = dmalloc(&P.desc, G, "desc")) ||
      (rc = dmalloc(&P.bbox_part, nc, "bbox")) ||
      (rc = dmalloc(&P.btotal, 1, "btotal")) || (rc = dmalloc(&P.keys, n, "keys")) ||
      (rc = dmalloc(&P.keys_tmp, n, "keys")) || (rc = dmalloc(&P.perm_tmp, n, "perm")) ||
      (rc = dmalloc(&P.perm_tmp2, n, "perm")) || (rc = dmalloc(&P.skeys, n, "keys")) ||
      (rc = dmalloc(&P.xs, n, "xs")) ||
      (rc = dmalloc(&P.bin_hist, ((size_t)1 << kBinDigitBits) * tiles, "hist")) ||
      (rc = dmalloc(&P.bin_rtot, (size_t)1 << kBinDigitBits, "hist")) ||
      (rc = dmalloc(&P.head_box, ranges, "ranges")) || (rc = dmalloc(&P.tail_box, ranges, "ranges")) ||
      (rc = dmalloc(&P.head_val, ranges * 27, "ranges")) ||
      (rc = dmalloc(&P.tail_val, ranges * 27, "ranges")) ||
      (rc = dmalloc(&P.perm, n, "perm")) || (rc = dmalloc(&P.rep_ent, n, "rep_ent")) ||
      (rc = dmalloc(&P.zi, n, "zi")) ||
      (rc = dmalloc(&P.lnv, n, "lnv")) || (rc = dmalloc(&P.slot_z, n, "slot_z")) ||
      (rc = dmalloc(&P.slot_ln, n, "slot_ln")) || (rc = dmalloc(&P.zpart, (size_t)nc * kGatherSplit, "zpart")) ||
      (rc = dmalloc(&P.zg, G, "zg")) || (rc = dmalloc(&P.cost_part, (size_t)nc * kCostTerms, "cost")))
    return rc;
  TSNET_HIP(hipMemcpy(P.ginfo, P.ginfo_h.data(), sizeof(GraphInfo) * G, hipMemcpyHostToDevice));
  TSNET_HIP(hipMemcpy(P.goff_d, P.goff.data(), sizeof(int) * (G + 1), hipMemcpyHostToDevice));
  if (G > 1) {  // graph of every vertex: one load instead of a search over the offsets
    std::vector<int> vg(n);
    for (int g = 0; g < G; ++g)
      for (int v = P.goff[g]; v < P.goff[g + 1]; ++v) vg[v] = g;
    if ((rc = dmalloc(&P.vgraph, n, "vgraph"))) return rc;
    TSNET_HIP(hipMemcpy(P.vgraph, vg.data(), sizeof(int) * n, hipMemcpyHostToDevice));
  }
  TSNET_HIP(hipMemcpy(P.chunk_graph, cg.data(), sizeof(int) * nc, hipMemcpyHostToDevice));
  TSNET_HIP(hipMemcpy(P.chunk_start, cs.data(), sizeof(int) * nc, hipMemcpyHostToDevice));
  TSNET_HIP(hipMemcpy(P.chunk_end, ce.data(), sizeof(int) * nc, hipMemcpyHostToDevice));
  TSNET_HIP(hipMemset(P.zg, 0, sizeof(double) * G));
  return TSNET_OK;
}

// Box offsets and far-point counts sized for `cap` boxes per axis in every
// graph; the grid buffers of a single graph sized for a cap x cap grid. A
// batch's grid buffers are pools sized from its plans (ensure_pools).
static int ensure_grid(Problem& P, int cap) {
  if (P.cap >= cap) return TSNET_OK;
  TSNET_HIP(hipDeviceSynchronize());
  free_grid(P);
  // every graph: cap^2 core boxes at most, then its far box
  const size_t boxes = (size_t)P.G * ((size_t)cap * cap + 1);
  if (boxes >= (size_t)1 << 30) return fail(TSNET_EINVAL, "too many interpolation boxes in batch");
  int rc;
  if ((rc = dmalloc(&P.box_off, boxes + 1, "box_off")) ||
      (rc = dmalloc(&P.trim_hist, (size_t)P.G * 2 * kTrimBins, "trim_hist"))) {
    free_grid(P);
    return rc;
  }
  void* h = nullptr;
  if (hipHostMalloc(&h, sizeof(size_t) * POOL_KINDS, hipHostMallocMapped) != hipSuccess || !h) {
    free_grid(P);
    return fail(TSNET_ENOMEM, "pinned host allocation failed (pool needs)");
  }
  P.need_host = static_cast<size_t*>(h);
  std::memset(P.need_host, 0, sizeof(size_t) * POOL_KINDS);
  void* hd = nullptr;
  if (hipHostGetDevicePointer(&hd, h, 0) != hipSuccess || !hd) {
    free_grid(P);
    return fail(TSNET_EHIP, "no device address for the pool needs");
  }
  P.need_dev = static_cast<size_t*>(hd);
  if (P.G == 1) {  // one graph: its pools hold the largest grid it may plan
    size_t c[POOL_KINDS];
    for (int k = 0; k < POOL_KINDS; ++k) c[k] = pool_elems(k, cap);
    if ((rc = alloc_pools(P, c))) {
      free_grid(P);
      return rc;
    }
  }
  TSNET_HIP(hipMemset(P.trim_hist, 0, sizeof(int) * (size_t)P.G * 2 * kTrimBins));
  P.cap = cap;
  return TSNET_OK;
}

// Layouts derived from P once it exists.
static int finish_problem(Problem& P, hipStream_t s) {
  if (P.nnz >= ((int64_t)1 << 31)) return fail(TSNET_EINVAL, "P has more than 2^31 nonzeros");
  int rc = build_row_order(P);
  if (!rc && P.n >= kTileAutoMinN && tiles_supported(P)) rc = build_tiles(P, s);
  return rc;
}

static bool use_tiles(const Problem& P, const tsnet_params& prm) {
  if (prm.attract_layout == TSNET_ATTRACT_TILED) return true;
  return prm.attract_layout == TSNET_ATTRACT_AUTO && P.n >= kTileAutoMinN && tiles_supported(P);
}

static int check_params(const tsnet_params* p) {
  if (!p) return fail(TSNET_EINVAL, "params is NULL");
  if (p->nodes_per_interval != kNodes) return fail(TSNET_EINVAL, "nodes_per_interval must be 3");
  const int mx = p->max_intervals, mn = p->min_intervals;
  if (mx < 1 || mx > kMaxIntervals || (mx & (mx - 1)))
    return fail(TSNET_EINVAL, "max_intervals must be a power of two in [1, 1024]");
  if (mn < 1 || mn > mx) return fail(TSNET_EINVAL, "min_intervals must be in [1, max_intervals]");
  if (p->far_trim < 0 || p->far_trim > kMaxFarTrim)
    return fail(TSNET_EINVAL, "far_trim must be in [0, 1024]");
  if (!(p->interval_width > 0) || !std::isfinite(p->interval_width))
    return fail(TSNET_EINVAL, "interval_width must be positive and finite");
  if (!(p->eps_r > 0) || !std::isfinite(p->eps_r)) return fail(TSNET_EINVAL, "eps_r must be > 0");
  if (!std::isfinite(p->lambda_kl) || !std::isfinite(p->lambda_c) || !std::isfinite(p->lambda_r))
    return fail(TSNET_EINVAL, "lambda values must be finite");
  if (p->attract_layout < TSNET_ATTRACT_AUTO || p->attract_layout > TSNET_ATTRACT_TILED)
    return fail(TSNET_EINVAL, "attract_layout must be 0, 1 or 2");
  if ((p->repulsion != TSNET_TERMS_INTERP && p->repulsion != TSNET_TERMS_QUADTREE) ||
      (p->entropy != TSNET_TERMS_INTERP && p->entropy != TSNET_TERMS_QUADTREE))
    return fail(TSNET_EINVAL, "repulsion and entropy must be TSNET_TERMS_INTERP or TSNET_TERMS_QUADTREE");
  if ((p->repulsion == TSNET_TERMS_QUADTREE || p->entropy == TSNET_TERMS_QUADTREE) &&
      !(p->theta > 0.0 && p->theta <= 0.7))
    return fail(TSNET_EINVAL, "theta must be in (0, 0.7] with a quadtree");
  return TSNET_OK;
}

static int check_call(tsnet_ctx ctx, tsnet_P P) {
  if (!ctx) return fail(TSNET_EINVAL, "ctx is NULL");
  if (!P) return fail(TSNET_EINVAL, "P is NULL");
  if (P->p.ctx != &ctx->c) return fail(TSNET_EINVAL, "P belongs to another context");
  if (!P->p.rowptr) return fail(TSNET_EINVAL, "P has no affinities");
  TSNET_HIP(hipSetDevice(ctx->c.device));
  (void)hipGetLastError();  // launch checks below report only this call's errors
  return TSNET_OK;
}

#define TSNET_LAUNCH(expr)                                                          \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) return fail(TSNET_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Pools of a batch's grid buffers. The first evaluation plans the grids of its
// layout once without a limit, waits for the plan and sizes every pool at
// four times what it needs (at most the size of max_intervals grids in every
// graph). Later evaluations read the needs the last finished plan left in
// mapped host memory (no wait) and grow the pools first when they fell
// short; the plan of an evaluation that finds them short halves its largest
// grids until they fit and raises TSNET_STATUS_WORKSPACE. Under stream
// capture nothing is waited for or allocated.
static int ensure_pools(Problem& P, const float2* X, const PlanParams& pp, bool may_trim,
                        hipStream_t s) {
  const bool have = P.pool_cap[0] > 0;
  bool grow = !have;
  if (have) {
    const volatile size_t* nh = P.need_host;
    for (int k = 0; k < POOL_KINDS; ++k) grow |= nh[k] > P.pool_cap[k];
  }
  if (!grow) return TSNET_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  TSNET_HIP(hipStreamIsCapturing(s, &cs));
  if (cs != hipStreamCaptureStatusNone) {
    if (!have)
      return fail(TSNET_EINVAL, "the first evaluation of a batch sizes its workspace and "
                                "cannot run under stream capture");
    return TSNET_OK;  // the plan fits the grids into the pools and flags it
  }
  if (!have) {
    PlanParams p0 = pp;
    for (int k = 0; k < POOL_KINDS; ++k) p0.cap[k] = SIZE_MAX;
    TSNET_LAUNCH(launch_bbox_plan(P, X, p0, may_trim, s));
    TSNET_LAUNCH(launch_trim_plan(P, X, p0, may_trim, s));
  }
  TSNET_HIP(hipStreamSynchronize(s));
  size_t cap[POOL_KINDS];
  for (int k = 0; k < POOL_KINDS; ++k) {
    const size_t full = pool_elems(k, P.cap) * (size_t)P.G;
    const size_t want = 4 * P.need_host[k];
    cap[k] = want < full ? want : full;
    if (cap[k] < P.need_host[k]) cap[k] = P.need_host[k];
  }
  TSNET_HIP(hipDeviceSynchronize());
  free_pools(P);
  return alloc_pools(P, cap);
}

// The interpolation pipeline shared by grad and cost: grid, sort, spread, FFT, gather.
static int run_interp(Problem& P, const float2* X, const tsnet_params& prm, int with_ln,
                      int with_zi, double* Z_out, hipStream_t s) {
  Ctx& c = *P.ctx;
  if (prm.max_intervals > kFftSmallM / (2 * kNodes) && !c.fft_large)
    return fail(TSNET_EINVAL, "max_intervals above 512 needs 75 KB of LDS per block, which this device does not give");
  int rc = ensure_grid(P, prm.max_intervals);
  if (rc) return rc;
  PlanParams pp{};
  pp.h_target = prm.interval_width;
  pp.min_int = prm.min_intervals;
  pp.max_int = prm.max_intervals;
  pp.far_trim = prm.far_trim;
  pp.need = P.need_dev;
  // far points need a graph of kTrimMinPoints vertices or more
  bool may_trim = false;
  for (const GraphInfo& g : P.ginfo_h) may_trim |= g.n >= kTrimMinPoints;
  may_trim = may_trim && prm.far_trim > 0;
  if (P.G > 1 && (rc = ensure_pools(P, X, pp, may_trim, s))) return rc;
  for (int k = 0; k < POOL_KINDS; ++k) pp.cap[k] = P.pool_cap[k];
  {
    StageScope t(c, ST_BBOX, s);
    TSNET_LAUNCH(launch_bbox_plan(P, X, pp, may_trim, s));
    TSNET_LAUNCH(launch_trim_plan(P, X, pp, may_trim, s));
  }
  {
    StageScope t(c, ST_BIN, s);
    TSNET_LAUNCH(launch_bin(P, X, s));
  }
  {
    StageScope t(c, ST_SPREAD, s);
    TSNET_LAUNCH(launch_spread(P, X, s));
  }
  {
    StageScope t(c, ST_FFT, s);
    TSNET_LAUNCH(launch_fft_conv(P, (float)prm.eps_r, with_ln, prm.max_intervals, s));
  }
  if (may_trim) {
    StageScope t(c, ST_FAR, s);
    TSNET_LAUNCH(launch_far(P, prm.far_trim, (float)prm.eps_r, with_ln, s));
  }
  {
    StageScope t(c, ST_GATHER, s);
    TSNET_LAUNCH(launch_gather(P, X, with_ln, with_zi, Z_out, s));
  }
  return TSNET_OK;
}

// The repulsion (with Z) and entropy sums by the methods prm selects: the
// interpolation fills all of them; a quadtree evaluation then replaces the
// ones it is chosen for (both: the interpolation is skipped).
static int run_terms(Problem& P, const float2* X, const tsnet_params& prm, int with_ln, int with_zi,
                     double* Z_out, hipStream_t s) {
  const bool qrep = prm.repulsion == TSNET_TERMS_QUADTREE;
  const bool qent = prm.entropy == TSNET_TERMS_QUADTREE;
  int rc;
  if (!qrep || !qent) {
    if ((rc = run_interp(P, X, prm, with_ln, with_zi, Z_out, s))) return rc;
  }
  if (qrep || qent) {
    const int terms = (qrep ? QT_REP : 0) | (qent ? QT_ENT : 0) | (qent && with_ln ? QT_LN : 0);
    StageScope t(*P.ctx, ST_QUADTREE, s);
    if ((rc = run_quadtree(P, X, prm.theta, (float)prm.eps_r, terms, qrep && with_zi,
                           qrep ? Z_out : nullptr, s)))
      return rc;
  }
  return TSNET_OK;
}

static int grad_impl(tsnet_ctx ctx, tsnet_P Pp, const float* X, const tsnet_params* prm, float* G,
                     double* Z_out, float* F_attr, float* F_rep, float* F_ent, float* Z_i,
                     void* stream) {
  int rc = check_call(ctx, Pp);
  if (rc) return rc;
  if ((rc = check_params(prm))) return rc;
  if (!X || !G) return fail(TSNET_EINVAL, "X and G must not be NULL");
  if ((const void*)X == (const void*)G) return fail(TSNET_EINVAL, "G may not alias X");
  Problem& P = Pp->p;
  Ctx& c = ctx->c;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const float2* X2 = reinterpret_cast<const float2*>(X);
  // the gather also reduces Z; Z_i is stored only when asked for
  if ((rc = run_terms(P, X2, *prm, 0, Z_i != nullptr, Z_out, s))) return rc;
  const bool tiled = use_tiles(P, *prm);
  if (tiled && P.tile_T == 0 && (rc = build_tiles(P, s))) return rc;
  {
    StageScope t(c, ST_ATTR, s);
    if (tiled)
      TSNET_LAUNCH(launch_attract_tiled(P, X2, *prm, reinterpret_cast<float2*>(G),
                                        reinterpret_cast<float2*>(F_attr), s));
    else
      TSNET_LAUNCH(launch_attract(P, X2, *prm, reinterpret_cast<float2*>(G),
                                  reinterpret_cast<float2*>(F_attr), s));
  }
  if (F_rep || F_ent || Z_i)
    TSNET_LAUNCH(launch_copy_terms(P, reinterpret_cast<float2*>(F_rep),
                                   reinterpret_cast<float2*>(F_ent), Z_i, s));
  return TSNET_OK;
}

}  // namespace tsnet

using namespace tsnet;

extern "C" {

void tsnet_default_params(tsnet_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->lambda_kl = 1.0;
  p->lambda_c = 1.2;
  p->lambda_r = 0.01;
  p->eps_r = 0.05;
  p->interval_width = 0.25;
  p->min_intervals = 50;
  p->max_intervals = 512;
  p->nodes_per_interval = 3;
  p->repulsion = TSNET_TERMS_INTERP;
  p->entropy = TSNET_TERMS_INTERP;
  p->theta = 0.5;
  p->far_trim = 64;
}

void tsnet_default_step_params(tsnet_step_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->eta = 0.0;
  p->momentum_early = 0.5;
  p->momentum_late = 0.8;
  p->min_gain = 0.01;
  p->gain_up = 0.2;
  p->gain_down = 0.8;
  p->momentum_switch_iter = 250;
}

int tsnet_ctx_create(tsnet_ctx* out, int device) {
  if (!out) return fail(TSNET_EINVAL, "out is NULL");
  *out = nullptr;
  int count = 0;
  TSNET_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(TSNET_EINVAL, "no such HIP device");
  TSNET_HIP(hipSetDevice(device));
  tsnet_ctx c = new (std::nothrow) tsnet_ctx_s;
  if (!c) return fail(TSNET_ENOMEM, "host allocation failed");
  c->c.device = device;
  std::vector<float2> tw(kMaxM);
  const double two_pi = 6.283185307179586476925286766559;
  for (int m = 0; m < kMaxM; ++m) {
    const double a = two_pi * (double)m / (double)kMaxM;
    tw[m] = make_float2((float)std::cos(a), (float)-std::sin(a));
  }
  int rc;
  if ((rc = dmalloc(&c->c.twiddle, kMaxM, "twiddle")) || (rc = dmalloc(&c->c.status, 1, "status"))) {
    dfree(c->c.twiddle);
    delete c;
    return rc;
  }
  hipError_t e = hipMemcpy(c->c.twiddle, tw.data(), sizeof(float2) * kMaxM, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(c->c.status, 0, sizeof(unsigned));
  if (e != hipSuccess) {
    dfree(c->c.twiddle);
    dfree(c->c.status);
    delete c;
    return fail(TSNET_EHIP, std::string("context set-up: ") + hipGetErrorString(e));
  }
  c->c.fft_large = fft_large_init();
  // the allocation-free direct call's scratch on this device (device current)
  if ((rc = static_scratch(device, &c->c.static_scratch))) {
    dfree(c->c.twiddle);
    dfree(c->c.status);
    delete c;
    return rc;
  }
  *out = c;
  return TSNET_OK;
}

int tsnet_ctx_destroy(tsnet_ctx ctx) {
  if (!ctx) return TSNET_OK;
  if (ctx->c.live_problems > 0)
    return fail(TSNET_EINVAL, "the context still owns problems: free them first");
  (void)hipSetDevice(ctx->c.device);
  (void)hipDeviceSynchronize();
  for (auto& p : ctx->c.pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : ctx->c.ev_free) (void)hipEventDestroy(e);
  dfree(ctx->c.twiddle);
  dfree(ctx->c.status);
  delete ctx;
  return TSNET_OK;
}

int tsnet_build_P(tsnet_ctx ctx, const int64_t* indptr, const int32_t* indices, int32_t n,
                  int64_t num_arcs, const int32_t* graph_offsets_host, int32_t num_graphs,
                  double perplexity, int32_t k, uint64_t tie_seed, int32_t tie_mode, tsnet_P* out,
                  void* stream) {
  if (!ctx || !out) return fail(TSNET_EINVAL, "ctx and out must not be NULL");
  *out = nullptr;
  if (!indptr || (num_arcs > 0 && !indices)) return fail(TSNET_EINVAL, "CSR pointers are NULL");
  if (n < 1) return fail(TSNET_EINVAL, "n must be >= 1");
  if (num_arcs < 0 || num_arcs >= ((int64_t)1 << 31)) return fail(TSNET_EINVAL, "bad num_arcs");
  if (!(perplexity > 0) || !std::isfinite(perplexity))
    return fail(TSNET_EINVAL, "perplexity must be positive and finite");
  if (k == 0) k = (int32_t)std::floor(3.0 * perplexity + 1e-9);
  if (k < 1 || k > kMaxK) return fail(TSNET_EINVAL, "k must be in [1, 1024]");
  if ((int64_t)n * k >= ((int64_t)1 << 31)) return fail(TSNET_EINVAL, "n * k too large");
  if (tie_mode != TSNET_TIE_HASH && tie_mode != TSNET_TIE_ID)
    return fail(TSNET_EINVAL, "unknown tie_mode");
  TSNET_HIP(hipSetDevice(ctx->c.device));
  tsnet_P P = new (std::nothrow) tsnet_P_s;
  if (!P) return fail(TSNET_ENOMEM, "host allocation failed");
  int rc = init_problem(ctx->c, P->p, n, graph_offsets_host, num_graphs);
  if (!rc) {
    P->p.k = k;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    StageScope t(ctx->c, ST_BUILD, s);
    rc = build_affinities(P->p, indptr, indices, num_arcs, perplexity, tie_seed, tie_mode, s);
    if (!rc) rc = finish_problem(P->p, s);
  }
  if (rc) {
    std::string msg = g_err;
    (void)hipDeviceSynchronize();
    free_problem(P->p);
    delete P;
    return fail(rc, msg);
  }
  *out = P;
  return TSNET_OK;
}

void tsnet_default_pmds_params(tsnet_pmds_params* p) {
  if (!p) return;
  p->pivots = 50;
  p->seed = 0;
  p->scale = 1e-2;
}

int tsnet_pmds(tsnet_ctx ctx, const int64_t* indptr, const int32_t* indices, int32_t n,
               int64_t num_arcs, const int32_t* graph_offsets_host, int32_t num_graphs,
               const tsnet_pmds_params* prm, float* X, int32_t* pivots, double* eig_host,
               int32_t* levels_host, void* stream) {
  if (!ctx || !prm || !X) return fail(TSNET_EINVAL, "ctx, params and X must not be NULL");
  if (!indptr || (num_arcs > 0 && !indices)) return fail(TSNET_EINVAL, "CSR pointers are NULL");
  if (n < 1) return fail(TSNET_EINVAL, "n must be >= 1");
  if (num_arcs < 0 || num_arcs >= ((int64_t)1 << 31)) return fail(TSNET_EINVAL, "bad num_arcs");
  if (prm->pivots < 1 || prm->pivots > 128) return fail(TSNET_EINVAL, "pivots must be in [1, 128]");
  if (!(prm->scale > 0) || !std::isfinite(prm->scale))
    return fail(TSNET_EINVAL, "scale must be positive and finite");
  if ((int64_t)std::min<int64_t>(prm->pivots, n) * n >= ((int64_t)1 << 31))
    return fail(TSNET_EINVAL, "n * pivots too large");
  std::vector<int> goff;
  int rc = check_offsets(n, graph_offsets_host, num_graphs, goff);
  if (rc) return rc;
  TSNET_HIP(hipSetDevice(ctx->c.device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int* goff_d = nullptr;
  TSNET_HIP(hipMalloc(reinterpret_cast<void**>(&goff_d), sizeof(int) * (num_graphs + 1)));
  hipError_t e = hipMemcpyAsync(goff_d, goff.data(), sizeof(int) * (num_graphs + 1),
                                hipMemcpyHostToDevice, s);
  rc = e != hipSuccess ? fail(TSNET_EHIP, hipGetErrorString(e))
                       : validate_csr(indptr, indices, n, num_arcs, goff_d, num_graphs, s);
  (void)hipStreamSynchronize(s);
  (void)hipFree(goff_d);
  if (rc) return rc;
  StageScope t(ctx->c, ST_PMDS, s);
  return run_pmds(indptr, indices, n, goff, prm->pivots, prm->seed, prm->scale, X, pivots,
                  eig_host, levels_host, s);
}

// Shared checks of the metric calls: pointers, sizes, offsets and the graph.
static int metric_graph(tsnet_ctx ctx, const int64_t* indptr, const int32_t* indices, int32_t n,
                        int64_t num_arcs, const int32_t* graph_offsets_host, int32_t num_graphs,
                        const float* X, std::vector<int>& goff, hipStream_t s) {
  if (!ctx || !X) return fail(TSNET_EINVAL, "ctx and X must not be NULL");
  if (!indptr || (num_arcs > 0 && !indices)) return fail(TSNET_EINVAL, "CSR pointers are NULL");
  if (n < 1) return fail(TSNET_EINVAL, "n must be >= 1");
  if (num_arcs < 0 || num_arcs >= ((int64_t)1 << 31)) return fail(TSNET_EINVAL, "bad num_arcs");
  int rc = check_offsets(n, graph_offsets_host, num_graphs, goff);
  if (rc) return rc;
  TSNET_HIP(hipSetDevice(ctx->c.device));
  int* goff_d = nullptr;
  TSNET_HIP(hipMalloc(reinterpret_cast<void**>(&goff_d), sizeof(int) * (num_graphs + 1)));
  hipError_t e = hipMemcpyAsync(goff_d, goff.data(), sizeof(int) * (num_graphs + 1),
                                hipMemcpyHostToDevice, s);
  rc = e != hipSuccess ? fail(TSNET_EHIP, hipGetErrorString(e))
                       : validate_csr(indptr, indices, n, num_arcs, goff_d, num_graphs, s);
  (void)hipStreamSynchronize(s);
  (void)hipFree(goff_d);
  return rc;
}

int tsnet_np(tsnet_ctx ctx, const int64_t* indptr, const int32_t* indices, int32_t n,
             int64_t num_arcs, const int32_t* graph_offsets_host, int32_t num_graphs,
             const float* X, const int32_t* vertices, int32_t num_vertices, int32_t* ball,
             int32_t* hits, double* np_host, void* stream) {
  if (!ball || !hits) return fail(TSNET_EINVAL, "ball and hits must not be NULL");
  if (vertices ? num_vertices < 1 : num_vertices != n)
    return fail(TSNET_EINVAL, "num_vertices must be >= 1, or n when vertices is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<int> goff;
  int rc = metric_graph(ctx, indptr, indices, n, num_arcs, graph_offsets_host, num_graphs, X, goff, s);
  if (rc) return rc;
  StageScope t(ctx->c, ST_NP, s);
  return run_np(indptr, indices, n, goff, X, vertices, num_vertices, ball, hits, np_host, s);
}

int tsnet_stress(tsnet_ctx ctx, const int64_t* indptr, const int32_t* indices, int32_t n,
                 int64_t num_arcs, const int32_t* graph_offsets_host, int32_t num_graphs,
                 const float* X, const int32_t* sources, int32_t num_sources, double* sums_host,
                 int32_t* levels_host, void* stream) {
  if (!sources || num_sources < 1) return fail(TSNET_EINVAL, "sources must name at least one vertex");
  if (!sums_host) return fail(TSNET_EINVAL, "sums_host must not be NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<int> goff;
  int rc = metric_graph(ctx, indptr, indices, n, num_arcs, graph_offsets_host, num_graphs, X, goff, s);
  if (rc) return rc;
  StageScope t(ctx->c, ST_STRESS, s);
  return run_stress(indptr, indices, n, goff, X, sources, num_sources, sums_host, levels_host, s);
}

int tsnet_P_from_host(tsnet_ctx ctx, int32_t n, const int64_t* rowptr_host,
                      const int32_t* col_host, const float* val_host,
                      const int32_t* graph_offsets_host, int32_t num_graphs, tsnet_P* out) {
  if (!ctx || !out) return fail(TSNET_EINVAL, "ctx and out must not be NULL");
  *out = nullptr;
  if (n < 1 || !rowptr_host) return fail(TSNET_EINVAL, "bad CSR");
  const int64_t nnz = rowptr_host[n];
  if (rowptr_host[0] != 0 || nnz < 0) return fail(TSNET_EINVAL, "bad rowptr");
  if (nnz > 0 && (!col_host || !val_host)) return fail(TSNET_EINVAL, "bad CSR");
  std::vector<int> goff;
  int rc = check_offsets(n, graph_offsets_host, num_graphs, goff);
  if (rc) return rc;
  for (int g = 0; g < num_graphs; ++g)
    for (int i = goff[g]; i < goff[g + 1]; ++i) {
      if (rowptr_host[i + 1] < rowptr_host[i]) return fail(TSNET_EINVAL, "rowptr not monotone");
      for (int64_t e = rowptr_host[i]; e < rowptr_host[i + 1]; ++e) {
        if (col_host[e] < goff[g] || col_host[e] >= goff[g + 1] || col_host[e] == i)
          return fail(TSNET_EINVAL, "column out of its graph or on the diagonal");
        if (!(val_host[e] >= 0.0f) || !std::isfinite(val_host[e]))
          return fail(TSNET_EINVAL, "P values must be finite and >= 0");
      }
    }
  TSNET_HIP(hipSetDevice(ctx->c.device));
  tsnet_P P = new (std::nothrow) tsnet_P_s;
  if (!P) return fail(TSNET_ENOMEM, "host allocation failed");
  rc = init_problem(ctx->c, P->p, n, graph_offsets_host, num_graphs);
  if (!rc) rc = dmalloc(&P->p.rowptr, (size_t)n + 1, "rowptr");
  if (!rc) rc = dmalloc(&P->p.col, (size_t)nnz, "col");
  if (!rc) rc = dmalloc(&P->p.val, (size_t)nnz, "val");
  if (!rc) {
    hipError_t e = hipMemcpy(P->p.rowptr, rowptr_host, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess && nnz > 0)
      e = hipMemcpy(P->p.col, col_host, sizeof(int) * nnz, hipMemcpyHostToDevice);
    if (e == hipSuccess && nnz > 0)
      e = hipMemcpy(P->p.val, val_host, sizeof(float) * nnz, hipMemcpyHostToDevice);
    if (e != hipSuccess) rc = fail(TSNET_EHIP, std::string("copy P: ") + hipGetErrorString(e));
  }
  if (!rc) {
    P->p.nnz = nnz;
    rc = finish_problem(P->p, nullptr);
  }
  if (rc) {
    std::string msg = g_err;
    free_problem(P->p);
    delete P;
    return fail(rc, msg);
  }
  P->p.nnz = nnz;
  *out = P;
  return TSNET_OK;
}

int tsnet_P_info(tsnet_P P, int64_t* n, int64_t* nnz, int32_t* num_graphs, int32_t* k) {
  if (!P) return fail(TSNET_EINVAL, "P is NULL");
  if (n) *n = P->p.n;
  if (nnz) *nnz = P->p.nnz;
  if (num_graphs) *num_graphs = P->p.G;
  if (k) *k = P->p.k;
  return TSNET_OK;
}

int tsnet_P_export(tsnet_P Pp, int64_t* rowptr, int32_t* col, float* val, double* beta,
                   int8_t* status, int32_t* cond_len, int32_t* cond_nbr, uint16_t* cond_dist) {
  if (!Pp) return fail(TSNET_EINVAL, "P is NULL");
  Problem& P = Pp->p;
  TSNET_HIP(hipSetDevice(P.ctx->device));
  TSNET_HIP(hipDeviceSynchronize());
  const bool want_cond = beta || status || cond_len || cond_nbr || cond_dist;
  if (want_cond && P.k == 0) return fail(TSNET_EINVAL, "P has no conditional rows");
  const size_t n = P.n, nk = (size_t)P.n * P.k;
  if (rowptr) TSNET_HIP(hipMemcpy(rowptr, P.rowptr, sizeof(int64_t) * (n + 1), hipMemcpyDefault));
  if (col && P.nnz) TSNET_HIP(hipMemcpy(col, P.col, sizeof(int) * P.nnz, hipMemcpyDefault));
  if (val && P.nnz) TSNET_HIP(hipMemcpy(val, P.val, sizeof(float) * P.nnz, hipMemcpyDefault));
  if (beta) TSNET_HIP(hipMemcpy(beta, P.beta, sizeof(double) * n, hipMemcpyDefault));
  if (status) TSNET_HIP(hipMemcpy(status, P.rstatus, n, hipMemcpyDefault));
  if (cond_len) TSNET_HIP(hipMemcpy(cond_len, P.cond_len, sizeof(int) * n, hipMemcpyDefault));
  if (cond_nbr) TSNET_HIP(hipMemcpy(cond_nbr, P.cond_nbr, sizeof(int) * nk, hipMemcpyDefault));
  if (cond_dist) TSNET_HIP(hipMemcpy(cond_dist, P.cond_dist, sizeof(uint16_t) * nk, hipMemcpyDefault));
  return TSNET_OK;
}

int tsnet_P_free(tsnet_P P) {
  if (!P) return TSNET_OK;
  (void)hipSetDevice(P->p.ctx->device);
  (void)hipDeviceSynchronize();
  free_problem(P->p);
  delete P;
  return TSNET_OK;
}

int tsnet_grad(tsnet_ctx ctx, tsnet_P P, const float* X, const tsnet_params* prm, float* G,
               double* Z_out, void* stream) {
  return grad_impl(ctx, P, X, prm, G, Z_out, nullptr, nullptr, nullptr, nullptr, stream);
}

int tsnet_grad_terms(tsnet_ctx ctx, tsnet_P P, const float* X, const tsnet_params* prm, float* G,
                     double* Z_out, float* F_attr, float* F_rep, float* F_ent, float* Z_i,
                     void* stream) {
  return grad_impl(ctx, P, X, prm, G, Z_out, F_attr, F_rep, F_ent, Z_i, stream);
}

int tsnet_step(tsnet_ctx ctx, tsnet_P Pp, float* X, float* update, float* gains, const float* G,
               const tsnet_step_params* sp, int32_t iter, void* stream) {
  int rc = check_call(ctx, Pp);
  if (rc) return rc;
  if (!X || !update || !gains || !G || !sp) return fail(TSNET_EINVAL, "NULL argument");
  if (iter < 0) return fail(TSNET_EINVAL, "iter must be >= 0");
  if (!std::isfinite(sp->eta) || !(sp->min_gain >= 0) || !std::isfinite(sp->momentum_early) ||
      !std::isfinite(sp->momentum_late) || !std::isfinite(sp->gain_up) || !std::isfinite(sp->gain_down))
    return fail(TSNET_EINVAL, "bad step parameters");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  StageScope t(ctx->c, ST_STEP, s);
  TSNET_LAUNCH(launch_step(Pp->p, reinterpret_cast<float2*>(X), reinterpret_cast<float2*>(update),
                           reinterpret_cast<float2*>(gains), reinterpret_cast<const float2*>(G), *sp,
                           iter, s));
  return TSNET_OK;
}

int tsnet_run(tsnet_ctx ctx, tsnet_P P, float* X, float* update, float* gains, float* G, double* Z,
              const tsnet_stage* stages, int32_t num_stages, int32_t first_iter,
              const tsnet_step_params* sp, void* stream) {
  int rc = check_call(ctx, P);
  if (rc) return rc;
  if (!stages || num_stages < 1) return fail(TSNET_EINVAL, "stages must hold at least one stage");
  if (first_iter < 0) return fail(TSNET_EINVAL, "first_iter must be >= 0");
  int64_t total = 0;
  for (int k = 0; k < num_stages; ++k) {
    if (stages[k].iterations < 0 || stages[k].reserved != 0)
      return fail(TSNET_EINVAL, "stage " + std::to_string(k) + ": iterations must be >= 0, reserved 0");
    if ((rc = check_params(&stages[k].params)))
      return fail(rc, "stage " + std::to_string(k) + ": " + g_err);
    total += stages[k].iterations;
  }
  if (first_iter + total > INT_MAX) return fail(TSNET_EINVAL, "too many iterations");
  int it = first_iter;
  for (int k = 0; k < num_stages; ++k)
    for (int i = 0; i < stages[k].iterations; ++i, ++it) {
      if ((rc = grad_impl(ctx, P, X, &stages[k].params, G, Z, nullptr, nullptr, nullptr, nullptr, stream)))
        return rc;
      if ((rc = tsnet_step(ctx, P, X, update, gains, G, sp, it, stream))) return rc;
    }
  return TSNET_OK;
}

int tsnet_cost(tsnet_ctx ctx, tsnet_P Pp, const float* X, const tsnet_params* prm, double* cost,
               void* stream) {
  int rc = check_call(ctx, Pp);
  if (rc) return rc;
  if ((rc = check_params(prm))) return rc;
  if (!X || !cost) return fail(TSNET_EINVAL, "X and cost must not be NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const float2* X2 = reinterpret_cast<const float2*>(X);
  if ((rc = run_terms(Pp->p, X2, *prm, 1, 0, nullptr, s))) return rc;
  StageScope t(ctx->c, ST_COST, s);
  TSNET_LAUNCH(launch_cost(Pp->p, X2, *prm, cost, s));
  return TSNET_OK;
}

int tsnet_grad_direct_f64(tsnet_ctx ctx, tsnet_P Pp, const double* X, const tsnet_params* prm,
                          double* G, double* Z_out, const int32_t* rows, int32_t nrows,
                          double* terms, void* stream) {
  int rc = check_call(ctx, Pp);
  if (rc) return rc;
  if (!prm || !std::isfinite(prm->eps_r) || !(prm->eps_r > 0))
    return fail(TSNET_EINVAL, "bad params");
  if (!X || !G) return fail(TSNET_EINVAL, "X and G must not be NULL");
  Problem& P = Pp->p;
  if (!rows) nrows = P.n;
  if (nrows < 1) return fail(TSNET_EINVAL, "nrows must be >= 1");
  const size_t need = ((size_t)(rows ? nrows : 0) + P.n) * 5;
  if (P.direct_part_len < need) {
    TSNET_HIP(hipDeviceSynchronize());
    dfree(P.direct_part);
    P.direct_part_len = 0;
    if ((rc = dmalloc(&P.direct_part, need, "direct scratch"))) return rc;
    P.direct_part_len = need;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  StageScope t(ctx->c, ST_DIRECT, s);
  TSNET_LAUNCH(launch_direct(P, reinterpret_cast<const double2*>(X), *prm,
                             reinterpret_cast<double2*>(G), Z_out, rows, nrows, terms,
                             P.direct_part, s));
  return TSNET_OK;
}

int tsnet_grad_direct_f64_static(tsnet_ctx ctx, tsnet_P Pp, const double* X,
                                 const tsnet_params* prm, double* G, double* Z_out,
                                 const int32_t* rows, int32_t nrows, double* terms, void* stream) {
  int rc = check_call(ctx, Pp);
  if (rc) return rc;
  if (!prm || !std::isfinite(prm->eps_r) || !(prm->eps_r > 0))
    return fail(TSNET_EINVAL, "bad params");
  if (!X || !G) return fail(TSNET_EINVAL, "X and G must not be NULL");
  Problem& P = Pp->p;
  if (!rows) nrows = P.n;
  if (nrows < 1) return fail(TSNET_EINVAL, "nrows must be >= 1");
  const size_t need = ((size_t)(rows ? nrows : 0) + P.n) * 5;
  if (need > kStaticScratchDoubles)
    return fail(TSNET_EINVAL, "5 (n + nrows) exceeds the 2^21 doubles of the static scratch");
  if (!ctx->c.static_scratch) return fail(TSNET_EHIP, "no static scratch on this device");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  TSNET_LAUNCH(launch_direct(P, reinterpret_cast<const double2*>(X), *prm,
                             reinterpret_cast<double2*>(G), Z_out, rows, nrows, terms,
                             ctx->c.static_scratch, s));
  return TSNET_OK;
}

int tsnet_grid_info(tsnet_P Pp, int32_t* n_intervals, float* box_side, float* x0, float* y0,
                    int32_t* far_points) {
  if (!Pp) return fail(TSNET_EINVAL, "P is NULL");
  Problem& P = Pp->p;
  if (!P.desc || !P.box_off) return fail(TSNET_EINVAL, "no grid yet");
  TSNET_HIP(hipSetDevice(P.ctx->device));
  TSNET_HIP(hipDeviceSynchronize());
  std::vector<GridDesc> d(P.G);
  TSNET_HIP(hipMemcpy(d.data(), P.desc, sizeof(GridDesc) * P.G, hipMemcpyDeviceToHost));
  for (int g = 0; g < P.G; ++g) {
    if (n_intervals) n_intervals[g] = d[g].n_int;
    if (box_side) box_side[g] = d[g].h;
    if (x0) x0[g] = d[g].x0;
    if (y0) y0[g] = d[g].y0;
    if (far_points) {
      int fo[2] = {0, 0};
      if (d[g].trimmed)
        TSNET_HIP(hipMemcpy(fo, P.box_off + far_key(d[g]), sizeof(int) * 2, hipMemcpyDeviceToHost));
      far_points[g] = fo[1] - fo[0];
    }
  }
  return TSNET_OK;
}

int tsnet_workspace_bytes(tsnet_P Pp, size_t* bytes_host) {
  if (!Pp || !bytes_host) return fail(TSNET_EINVAL, "NULL argument");
  const Problem& P = Pp->p;
  const size_t per[POOL_KINDS] = {sizeof(float), 2 * sizeof(float2), 2 * sizeof(float),
                                  2 * sizeof(float2), sizeof(float)};  // q, k, o: two arrays each
  size_t b = 0;
  for (int k = 0; k < POOL_KINDS; ++k) b += P.pool_cap[k] * per[k];
  if (P.cap > 0) {
    b += sizeof(int) * ((size_t)P.G * ((size_t)P.cap * P.cap + 1) + 1);  // box offsets
    b += sizeof(int) * (size_t)P.G * 2 * kTrimBins;                     // far-point bin counts
  }
  *bytes_host = b;
  return TSNET_OK;
}

int tsnet_status(tsnet_ctx ctx, uint32_t* flags_host) {
  if (!ctx || !flags_host) return fail(TSNET_EINVAL, "NULL argument");
  TSNET_HIP(hipSetDevice(ctx->c.device));
  TSNET_HIP(hipDeviceSynchronize());
  unsigned v = 0;
  TSNET_HIP(hipMemcpy(&v, ctx->c.status, sizeof(unsigned), hipMemcpyDeviceToHost));
  TSNET_HIP(hipMemset(ctx->c.status, 0, sizeof(unsigned)));
  *flags_host = v;
  return TSNET_OK;
}

int tsnet_set_timing(tsnet_ctx ctx, uint32_t stage_mask) {
  if (!ctx) return fail(TSNET_EINVAL, "ctx is NULL");
  ctx->c.timing = stage_mask & ((1u << ST_COUNT) - 1u);
  return TSNET_OK;
}

int tsnet_stage_count(void) { return ST_COUNT; }

const char* tsnet_stage_name(int stage) {
  if (stage < 0 || stage >= ST_COUNT) return "";
  return kStageNames[stage];
}

int tsnet_stage_times(tsnet_ctx ctx, double* ms_host, int64_t* calls_host) {
  if (!ctx) return fail(TSNET_EINVAL, "ctx is NULL");
  TSNET_HIP(hipSetDevice(ctx->c.device));
  int rc = collect_times(ctx->c);
  if (rc) return rc;
  for (int i = 0; i < ST_COUNT; ++i) {
    if (ms_host) ms_host[i] = ctx->c.stage_ms[i];
    if (calls_host) calls_host[i] = ctx->c.stage_calls[i];
    ctx->c.stage_ms[i] = 0.0;
    ctx->c.stage_calls[i] = 0;
  }
  return TSNET_OK;
}

const char* tsnet_last_error(void) { return g_err.c_str(); }

}  // extern "C"
