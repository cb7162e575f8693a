// Internal declarations shared by the host ABI code and the HIP kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "tsnet.h"

namespace tsnet {

// ---------------------------------------------------------------- constants
constexpr int kNodes = 3;                 // interpolation nodes per box and axis
constexpr int kMaxIntervals = 1024;       // boxes per axis (power of two)
constexpr int kFftSmallM = 3072;          // FFT lengths of the small transform class (512 intervals)
constexpr int kMaxNg = kNodes * kMaxIntervals;
constexpr int kMaxM = 2 * kMaxNg;         // FFT length per axis (3 * 2^b)
constexpr int kPotCh = 8;                 // potential channels per node (4 planes of pairs)
constexpr int kCostTerms = 4;             // chunk sums of the cost reduction
constexpr int kSpreadRange = 1024;        // sorted points per wave in the spread (at most)
constexpr int kGatherSplit = 4;           // gather blocks per chunk
constexpr int kChunk = 2048;              // vertices per chunk of per-vertex kernels
constexpr int kMaxK = 1024;               // neighbours per vertex in tsnet_build_P
constexpr double kSpanFloor = 1e-4;       // smallest grid span (degenerate layouts)
constexpr int kBinTileH = 2048;           // points per tile of the binning radix sort
constexpr int kBinDigitBits = 10;         // digit width of the binning radix sort
constexpr int kRadixTile = 2048;          // elements per block tile of the LSD radix sort
constexpr int kTileMaxRows = 4096;        // rows per row tile of the tiled attraction
constexpr int kTileSlotBits = 12;         // bits of a row slot inside a tile
constexpr int kTileMinTiles = 256;        // row tiles (one workgroup each) at least
constexpr int kTileAutoMinN = 262144;     // automatic layout: tiled from this many vertices
constexpr int kTrimBins = 2048;           // bins per axis of the far-point rule
constexpr int kTrimMinPoints = 64;        // points per far point allowed (t <= n / 64)
constexpr int kMaxFarTrim = 1024;         // largest far_trim accepted
constexpr size_t kStaticScratchDoubles = (size_t)1 << 21;  // scratch of the allocation-free direct call

// Output channels of the convolution (charge index in comments):
//  0 K2*1, 1 K2*x, 2 K2*y, 3 K1*1, 4 Ke*1, 5 Ke*x, 6 Ke*y, 7 Kln*1
enum { CH_K2_1 = 0, CH_K2_X, CH_K2_Y, CH_K1_1, CH_KE_1, CH_KE_X, CH_KE_Y, CH_KLN_1 };

// Per-graph interpolation grid, rewritten on the device every evaluation.
// The grid covers the bounding box, or the core region when far points are
// set apart (trimmed = 1): a point is far when its bin on either axis lies
// outside [lo, hi], bin = min(floor((v - v_min) * s), kTrimBins - 1) in FP64.
// Box ids of the graph: n_int^2 core boxes from box_base, then its far box.
struct GridDesc {
  float x0, y0;      // lower-left corner of the box grid
  float h, inv_h;    // box side and its inverse
  float cx, cy;      // charge centre (centre of the covered region)
  float half;        // half the grid side: charges x, y are stored divided by it
  float spacing;     // node spacing h / 3
  int n_int;         // boxes per axis
  int ng;            // nodes per axis (3 n_int)
  int M;             // FFT length per axis (2 ng)
  int box_base;      // first global box id of this graph
  int flags;         // TSNET_STATUS_* bits raised by this graph
  int trimmed;       // 1: far points set apart (bounding-box kernel: 1 = may be)
  int trim_t;        // t = min(far_trim, n / kTrimMinPoints)
  int lo_x, hi_x, lo_y, hi_y;  // core bins per axis
  float bmin_x, bmin_y;        // bounding box of the graph's points
  float bmax_x, bmax_y;
  int pad0;
  double s_x, s_y;   // kTrimBins / width per axis (0 for a zero width)
  // element offsets of the graph's grid buffers in the workspace pools
  size_t off_c;      // charges (float, 3 ng^2)
  size_t off_q;      // charge row spectra and their transposes (float2, 3 ng Mh)
  size_t off_k;      // kernel spectra and their transposes (float, 4 Mh^2)
  size_t off_o;      // products and their transposes (float2, 8 ng Mh)
  size_t off_p;      // potentials (float, 8 ng^2)
};

// Workspace pool kinds, in the order of GridDesc's offsets.
enum { POOL_C = 0, POOL_Q, POOL_K, POOL_O, POOL_P, POOL_KINDS };

// Elements of each pool kind one graph with n_int boxes per axis needs
// (rounded up to 64 elements, so every graph's part starts 256-byte aligned).
__host__ __device__ inline size_t pool_elems(int kind, int n_int) {
  const size_t ng = 3 * (size_t)n_int, mh = ng + 1;
  size_t e = 0;
  switch (kind) {
    case POOL_C: e = 3 * ng * ng; break;
    case POOL_Q: e = 3 * ng * mh; break;
    case POOL_K: e = 4 * mh * mh; break;
    case POOL_O: e = 8 * ng * mh; break;
    default: e = 8 * ng * ng; break;
  }
  return (e + 63) & ~(size_t)63;
}

__host__ __device__ inline int far_key(const GridDesc& d) { return d.box_base + d.n_int * d.n_int; }

// Static per-graph data (device copy made once per problem).
struct GraphInfo {
  int vstart;        // first vertex
  int n;             // vertices
  int chunk_begin;   // first chunk of per-vertex kernels
  int chunk_end;
  float inv_n;       // 1 / n
  float inv_n2;      // 1 / n^2
  float lr;          // default learning rate max(200, n / 12)
  int pad;
};

struct PlanParams {
  double h_target;
  int min_int, max_int;
  int far_trim;      // t of the far-point rule (0: the grid covers the bounding box)
  int pad;
  size_t cap[POOL_KINDS];  // pool capacities in elements (SIZE_MAX: no limit)
  size_t* need;            // mapped host memory: the plan's pool needs, before any capping
};

// Stage ids for optional per-stage timing.
enum Stage {
  ST_BBOX = 0, ST_BIN, ST_SPREAD, ST_FFT, ST_GATHER, ST_ZRED, ST_ATTR, ST_STEP, ST_COST,
  ST_DIRECT, ST_BUILD, ST_PMDS, ST_NP, ST_STRESS, ST_QUADTREE, ST_FAR, ST_COUNT
};

// ---------------------------------------------------------------- contexts
struct Ctx {
  int device = 0;
  float2* twiddle = nullptr;          // e^{-2 pi i m / kMaxM}, m < kMaxM
  bool fft_large = false;             // grids of 1024 intervals available on this device
  double* static_scratch = nullptr;   // this device's scratch array of the allocation-free call
  unsigned* status = nullptr;         // device status word
  int lds_per_block = 65536;
  uint32_t timing = 0;                // bit s: time stage s
  int live_problems = 0;              // problems made in this context and not yet freed
  std::vector<hipEvent_t> ev_free;    // recycled events
  struct Pending { int stage; hipEvent_t a, b; };
  std::vector<Pending> pending;
  double stage_ms[ST_COUNT] = {0};
  int64_t stage_calls[ST_COUNT] = {0};
};

struct QuadWs;  // quadtree workspace (quadtree.hip), allocated on first use

struct Problem {
  Ctx* ctx = nullptr;
  int n = 0;
  int G = 0;
  int k = 0;                          // 0 for problems made from host CSR
  int64_t nnz = 0;
  std::vector<int> goff;              // host graph offsets [G+1]
  std::vector<GraphInfo> ginfo_h;
  int num_chunks = 0;
  // device: graph data
  GraphInfo* ginfo = nullptr;
  int* goff_d = nullptr;              // [G+1]
  int* vgraph = nullptr;              // [n] graph of every vertex (batches only)
  int* chunk_graph = nullptr;         // [num_chunks]
  int* chunk_start = nullptr;
  int* chunk_end = nullptr;
  // device: P (CSR)
  int64_t* rowptr = nullptr;
  int* col = nullptr;
  float* val = nullptr;
  int* row_order = nullptr;           // [n] rows by decreasing length (attraction order)
  int attract_blocks = 0;             // blocks of the row attraction the device holds at once
  // device: tiled copy of P for the attraction (row tiles x column windows)
  int tile_T = 0, tile_R = 0;         // row tiles, slots per tile
  int64_t tile_NB = 0;                // blocks (tile, column window) in all
  int* tile_rows = nullptr;           // [T * R] vertex of each slot, -1 if unused
  int* tile_wlo = nullptr;            // [T] first column window of each tile
  int* tile_boff = nullptr;           // [T + 1] first block of each tile
  int* tile_graph = nullptr;          // [T] graph of each tile's rows
  int* tile_order = nullptr;          // [T] tile of each block (largest tiles first)
  int* tile_bstart = nullptr;         // [NB + 1] first entry of each block
  uint2* tile_ent = nullptr;          // [nnz] {slot << 13 | column in window, value bits}
  // device: conditional rows and calibration (absent for host-made P)
  double* beta = nullptr;
  int8_t* rstatus = nullptr;
  int* cond_len = nullptr;
  int* cond_nbr = nullptr;
  uint16_t* cond_dist = nullptr;
  // device: per-evaluation workspace
  int cap = 0;                        // max_intervals the grid buffers are sized for
  GridDesc* desc = nullptr;           // [G]
  float4* bbox_part = nullptr;        // [num_chunks]
  int* btotal = nullptr;              // [1] total boxes of the batch
  int* keys = nullptr;                // [n] box id of every vertex
  int* keys_tmp = nullptr;            // [n] radix ping-pong
  int* perm_tmp = nullptr;            // [n]
  int* perm_tmp2 = nullptr;           // [n]
  int* skeys = nullptr;               // [n] box ids in sorted order
  int* perm = nullptr;                // [n] vertex of each sorted slot
  float2* xs = nullptr;               // [n] X in sorted order
  int* bin_hist = nullptr;            // [kDigits][tiles] digit counts, then their row prefixes
  int* bin_rtot = nullptr;            // [kDigits] digit totals of the current binning pass
  int* box_off = nullptr;             // [G (cap^2 + 1) + 1] first sorted slot of every box
  int* trim_hist = nullptr;           // [G][2][kTrimBins] bin counts (kept at zero between calls)
  float* slot_z = nullptr;            // [n] Z_i of far points, by sorted slot
  float* slot_ln = nullptr;           // [n] interpolated ln sums of far points, by sorted slot
  // grid buffers: one pool per kind, each graph at its own offset (GridDesc)
  float* charges = nullptr;           // per graph 3 ng^2
  float2* qspec = nullptr;            // per graph [3][ng][M/2+1] row spectra of the charges
  float2* qspec_t = nullptr;          // per graph [3][M/2+1][ng] the same, transposed
  float* kspec = nullptr;             // per graph [4][M/2+1][M/2+1] row spectra of the kernels
  float* kspec_t = nullptr;           // per graph the same, transposed
  float2* ospec_t = nullptr;          // per graph [8][M/2+1][ng] products after the column stage
  float2* ospec = nullptr;            // per graph [8][ng][M/2+1] the same, transposed
  float* pot = nullptr;               // per graph 4 planes (channel pairs) of ng^2 float2
  size_t pool_cap[POOL_KINDS] = {0, 0, 0, 0, 0};  // capacities in elements (0: not allocated)
  size_t* need_host = nullptr;        // pinned, mapped: the latest plan's needs [POOL_KINDS]
  size_t* need_dev = nullptr;         // its device address
  int spread_range = kSpreadRange;    // sorted points per wave of the spread (64 .. kSpreadRange)
  int* head_box = nullptr;            // [spread ranges] box of the leading partial, -1 if none
  int* tail_box = nullptr;            // [spread ranges] box of the trailing partial, -1 if none
  float* head_val = nullptr;          // [spread ranges][27]
  float* tail_val = nullptr;          // [spread ranges][27]
  float4* rep_ent = nullptr;          // [n] (F_rep.x, F_rep.y, F_ent.x, F_ent.y) of each vertex
  float* zi = nullptr;                // [n]
  float* lnv = nullptr;               // [n] interpolated sum_j ln(eps + r^2) (cost path)
  double* zpart = nullptr;            // [num_chunks * kGatherSplit] Z sums of the gather's parts
  double* zg = nullptr;               // [G]
  double* cost_part = nullptr;        // [num_chunks * 5]
  double* direct_part = nullptr;      // scratch of the FP64 direct kernel
  size_t direct_part_len = 0;
  QuadWs* qt = nullptr;               // quadtree sums (repulsion / entropy by quadtree)
};

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
#define TSNET_HIP(call)                                                            \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::tsnet::fail(TSNET_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------- launchers
// Every launcher enqueues on `s` and returns hipGetLastError().

// per-evaluation path (iter.hip, bin.hip, attract.hip)
hipError_t launch_bbox_plan(Problem& P, const float2* X, const PlanParams& pp, bool with_hist,
                            hipStream_t s);
// `pp` carries the pool capacities; the plan writes the uncapped needs to pp.need
// far-point rule: bin counts (only when some graph may set points apart), then the grid plan
hipError_t launch_trim_plan(Problem& P, const float2* X, const PlanParams& pp, bool with_hist,
                            hipStream_t s);
// far points: their own sums from the node charges and each other, and their
// charges added to the node potentials (between the FFT and the gather)
hipError_t launch_far(Problem& P, int far_trim, float eps, int with_ln, hipStream_t s);
hipError_t launch_bin(Problem& P, const float2* X, hipStream_t s);
hipError_t launch_spread(Problem& P, const float2* X, hipStream_t s);
// gather also reduces Z per graph into zg (and Z_out when not NULL)
hipError_t launch_gather(Problem& P, const float2* X, int with_ln, int with_zi, double* Z_out,
                         hipStream_t s);
hipError_t launch_attract(Problem& P, const float2* X, const tsnet_params& prm, float2* G,
                          float2* F_attr, hipStream_t s);
hipError_t launch_attract_tiled(Problem& P, const float2* X, const tsnet_params& prm, float2* G,
                                float2* F_attr, hipStream_t s);
hipError_t launch_step(Problem& P, float2* X, float2* upd, float2* gains, const float2* G,
                       const tsnet_step_params& sp, int iter, hipStream_t s);
hipError_t launch_cost(Problem& P, const float2* X, const tsnet_params& prm, double* cost,
                       hipStream_t s);
hipError_t launch_copy_terms(Problem& P, float2* F_rep, float2* F_ent, float* Z_i, hipStream_t s);

// visiting order of the attraction rows (attract.hip), built once per problem
int build_row_order(Problem& P);

// tiled copy of P for the attraction (tile.hip), built once per problem
bool tiles_supported(const Problem& P);
int build_tiles(Problem& P, hipStream_t s);

// stable LSD radix sort of (key, value) pairs by the low `bits` key bits, 8-bit
// digits (build.hip); the result ends in (keys, vals); kt, vt are N-entry
// ping-pong buffers, hist needs 256 * ceil(N / kRadixTile) + 1 ints, tsum the
// scan scratch of that length.
hipError_t radix_sort(unsigned* keys, unsigned* vals, unsigned* kt, unsigned* vt, int N, int bits,
                      int* hist, int* tsum, hipStream_t s);

// FFT convolution (fft.hip)
hipError_t launch_fft_conv(Problem& P, float eps, int with_ln, int max_intervals, hipStream_t s);
// Enables the transform class for 1024 intervals on the current device (false: not available).
bool fft_large_init();

// direct FP64 baseline (direct.hip); the pair sums go to `pairs`, which holds
// (n + nrows) * 5 doubles with rows, n * 5 without
hipError_t launch_direct(Problem& P, const double2* X, const tsnet_params& prm, double2* G,
                         double* Z_out, const int* rows, int nrows, double* terms, double* pairs,
                         hipStream_t s);
// device address of the allocation-free direct call's scratch array on `device`
// (looked up once per device; synchronous)
int static_scratch(int device, double** out);

// Pivot MDS starting layout (pmds.hip). goff: host graph offsets [G+1].
// Synchronous; X [n][2] on the device, pivots_out [G][pivots] device or NULL,
// eig_host [G][2] or NULL, levels_host: BFS levels run (or NULL).
int run_pmds(const int64_t* indptr, const int* indices, int n, const std::vector<int>& goff,
             int pivots, uint64_t seed, double scale, float* X, int* pivots_out, double* eig_host,
             int* levels_host, hipStream_t s);

// Barnes-Hut quadtree sums (quadtree.hip): the tree is rebuilt from X and
// each point's sums are written where the interpolation puts them: QT_REP
// fills rep_ent.xy, the per-vertex z (into zi when with_zi) and Z per graph
// (zg, and Z_out when not NULL); QT_ENT fills rep_ent.zw; QT_LN fills lnv
// (with the self term ln(eps), as the gather does).
// Enqueues only (no host synchronisation), so it may be captured.
enum { QT_REP = 1, QT_ENT = 2, QT_LN = 4 };
void free_quadtree(Problem& P);
int run_quadtree(Problem& P, const float2* X, double theta, float eps, int terms, int with_zi,
                 double* Z_out, hipStream_t s);

// layout quality metrics (metrics.hip); synchronous. Neighbourhood preservation:
// verts (device, strictly increasing) or NULL for all n, ball/hits [nv] on the
// device, np_host [G]. Stress: sources [nsrc] on the device, sums_host [G][6].
int run_np(const int64_t* indptr, const int* indices, int n, const std::vector<int>& goff,
           const float* X, const int* verts, int nv, int* ball, int* hits, double* np_host,
           hipStream_t s);
int run_stress(const int64_t* indptr, const int* indices, int n, const std::vector<int>& goff,
               const float* X, const int* sources, int nsrc, double* sums_host, int* levels_host,
               hipStream_t s);

// affinity build (build.hip)
// Checks a device CSR graph batch (row pointers, ranges, order, symmetry, no self loops or
// edges between graphs); TSNET_EINVAL with the reason otherwise. Synchronous.
int validate_csr(const int64_t* indptr, const int* indices, int n, int64_t num_arcs,
                 const int* goff_d, int G, hipStream_t s);
int build_affinities(Problem& P, const int64_t* indptr, const int* indices, int64_t num_arcs,
                     double perplexity, uint64_t seed, int tie_mode, hipStream_t s);

}  // namespace tsnet
