// Attractive KL term (Eq. 6, first sum) over a two-dimensional tiling of P,
// fused with the gradient assembly
//   G_i = 4 l_kl (F_attr,i - F_rep,i / Z) + (l_c / n) X_i - (l_r / n^2) F_ent,i.
//
// The row-parallel kernel (attract.hip) gathers x_j straight from HBM; on a
// graph like Barabasi-Albert the columns of a row are scattered over all of X,
// so most of those gathers miss L2 and refetch whole lines. Here the gathers
// come from LDS instead:
//
//  * the rows of each graph are dealt to the graph's row tiles in snake order
//    over decreasing row length (every tile of a graph holds about the same
//    number of entries); the rows of a tile get slots 0 .. R-1;
//  * columns are cut into windows of kTileCols vertices; a tile spans the
//    windows that its graph's vertices fall in (P is block-diagonal over the
//    graphs of a batch, so no entry of a tile lies outside them);
//  * block (t, c) holds the entries of tile t's rows whose column lies in
//    the tile's c-th window, ordered by slot and packed as {slot << 13 |
//    column offset in the window, value bits}.
//
// One workgroup per row tile walks its windows in order, with X[window] in LDS
// (the next window is fetched into registers while the current one is in use)
// and the row sums of its tile in LDS. A block is cut into 16 equal pieces,
// one per wave; a lane walks a run of up to 6 consecutive entries, and partial
// row sums are joined across lanes by a segmented scan. A row that continues
// from the previous wave's piece is parked in a slot of its own and added once
// the window is done. Every sum is taken in an order fixed by the layout, so
// results are reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <initializer_list>
#include <numeric>
#include <string>
#include <vector>

#include "dev_util.h"
#include "scan.h"
#include "tsnet_internal.h"

namespace tsnet {

constexpr int kTileColBits = 13;
constexpr int kTileCols = 1 << kTileColBits;  // vertices per column window (64 KB of X)
constexpr int kTileThreads = 1024;
constexpr int kTileWaves = kTileThreads / kWave;
constexpr int kTileRun = 6;                   // entries per lane and pass
constexpr int kTileNone = 0x7fffffff;         // key of a lane without entries
constexpr int kTileMaxNC = 768;               // column windows at most (block starts in LDS)

static_assert(kTileMaxRows <= (1 << kTileSlotBits), "slot field too narrow");
static_assert(kTileSlotBits + kTileColBits <= 32, "packed entry too wide");

struct TileArgs {
  const float2* X;
  int n, R;
  int last;               // nnz - 1 (at least 0: the entry array has one element or more)
  const int* tile_rows;   // [T * R] vertex of each slot, -1 for an unused slot
  const int* wlo;         // [T] first column window of each tile
  const int* boff;        // [T + 1] first block of each tile
  const int* tgraph;      // [T] graph of each tile
  const int* order;       // [T] tile of each block: tiles by decreasing entry count
  const int* bstart;      // [NB + 1] first entry of every block
  const uint2* ent;       // [nnz]
  const GraphInfo* gi;
  const double* zg;
  const float4* rep_ent;  // (F_rep, F_ent) of each vertex
  float lkl4, lc, lr;
  float2* Gout;
  float2* Fattr;
};

// Entries [p0, p1) of wave `wv` in window c of the tile (bst: the tile's
// block starts, in LDS). A row continues from the previous piece when the
// entries at p0 - 1 and p0 share a slot; both are fetched with the piece
// (indices clamped into the array, so every load is unconditional and the
// compiler can keep them in flight) and compared when it is used.
struct Piece {
  int bs, p0, p1;
  unsigned at, before;  // packed words of entries p0 and p0 - 1
};

__device__ __forceinline__ Piece piece_of(const TileArgs& a, const int* bst, int c, int wv) {
  const int bs = bst[c], be = bst[c + 1];
  const int64_t L = be - bs;
  Piece p;
  p.bs = bs;
  p.p0 = bs + (int)((L * wv) / kTileWaves);
  p.p1 = bs + (int)((L * (wv + 1)) / kTileWaves);
  p.at = a.ent[min(p.p0, a.last)].x;
  p.before = a.ent[max(0, min(p.p0 - 1, a.last))].x;
  return p;
}

// Slot of a row that began in the previous wave's piece, else -1.
__device__ __forceinline__ int piece_head(const Piece& p) {
  const unsigned s0 = p.at >> kTileColBits, sm = p.before >> kTileColBits;
  return p.p0 > p.bs && p.p0 < p.p1 && s0 == sm ? (int)s0 : -1;
}

__device__ __forceinline__ void run_of(int base, int p1, int lane, int& s0, int& cnt) {
  const int Lp = min(kWave * kTileRun, p1 - base);
  const int U = (Lp + kWave - 1) / kWave;
  s0 = base + lane * U;
  cnt = max(0, min(U, base + Lp - s0));
}

// Vertex of slot q * kTileThreads + tid of tile t for every q, -1 where the
// slot is unused or beyond R (loads clamped into the tile, none conditional).
constexpr int kTileRowsPerThread = kTileMaxRows / kTileThreads;
__device__ __forceinline__ void tile_row_ids(const TileArgs& a, int t, int tid,
                                             int (&iv)[kTileRowsPerThread]) {
#pragma unroll
  for (int q = 0; q < kTileRowsPerThread; ++q) {
    const int s = q * kTileThreads + tid;
    iv[q] = a.tile_rows[(size_t)t * a.R + min(s, a.R - 1)];
    if (s >= a.R) iv[q] = -1;
  }
}

struct Carry {
  int row;      // slot carried into the next pass, -1 if none
  float x, y;
};

// Adds a finished row sum: into the tile accumulator, or into the wave's
// parking slot when the row began in the previous wave's piece.
__device__ __forceinline__ void flush(int row, float x, float y, int head, int wv, float4* rec,
                                      int* hrow, float2* hval) {
  if (row == head) {
    hrow[wv] = row;
    hval[wv] = make_float2(x, y);
  } else {
    float2* acc = reinterpret_cast<float2*>(&rec[row].z);
    float2 v = *acc;
    v.x += x;
    v.y += y;
    *acc = v;
  }
}

// One step of the segmented inclusive scan: add the partial sums that the
// move brings in when they belong to the same slot (keys are sorted along
// the wave, so equal end points mean one segment).
template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_step(int key, float& sx, float& sy) {
  const int kk = dpp_i<CTRL, ROWS>(kTileNone - 1, key);
  const float ax = dpp_f<CTRL, ROWS>(0.f, sx), ay = dpp_f<CTRL, ROWS>(0.f, sy);
  if (kk == key) {
    sx += ax;
    sy += ay;
  }
}

// One pass over up to 64 * kTileRun consecutive entries of a piece. Lane l
// takes a run of cnt consecutive entries (sorted by slot). Its contributions
// are summed per slot in order; a slot that starts and ends inside the lane
// is added to the tile accumulator at once, the lane's first and last slots
// go through the scan across lanes below.
__device__ __forceinline__ void tile_pass(const uint2 (&e)[kTileRun], int cnt, bool more, int lane,
                                          int wv, int head, const float2* win, float4* rec,
                                          int* hrow, float2* hval, Carry& cr) {
  int r[kTileRun];
  float4 ri[kTileRun];  // (x_i, sum so far) of the entry's row: one 16-byte read
  float2 xj[kTileRun];
#pragma unroll
  for (int k = 0; k < kTileRun; ++k) {  // all LDS reads in flight together
    r[k] = (int)(e[k].x >> kTileColBits);
    ri[k] = rec[r[k]];
    xj[k] = win[e[k].x & (kTileCols - 1)];
  }
  const int r0 = r[0];
  int rl = r0;
#pragma unroll
  for (int k = 1; k < kTileRun; ++k)
    if (k < cnt) rl = r[k];
  float cx = 0.f, cy = 0.f, fx = 0.f, fy = 0.f;
  float2 own[kTileRun];  // sums of the slots wholly inside this lane
  bool put[kTileRun];
#pragma unroll
  for (int k = 0; k < kTileRun; ++k) {
    const float dx = ri[k].x - xj[k].x, dy = ri[k].y - xj[k].y;
    const float w = __uint_as_float(e[k].y) * __builtin_amdgcn_rcpf(1.0f + dx * dx + dy * dy);
    const bool valid = k < cnt;
    const bool same = k > 0 && r[k] == r[k - 1];
    const float wx = w * dx, wy = w * dy;
    if (valid) {
      cx = same ? cx + wx : wx;
      cy = same ? cy + wy : wy;
    }
    const bool ends = valid && (k + 1 >= cnt || (k + 1 < kTileRun && r[k + 1] != r[k]));
    if (ends && r[k] == r0) {
      fx = cx;
      fy = cy;
    }
    put[k] = ends && r[k] != r0 && r[k] != rl;
    own[k] = make_float2(cx, cy);
  }
  // no other lane or wave touches those slots in this window, so the sums
  // read with x_i above are current (slots of the clamped tail entries are
  // valid indices and are read but not written)
#pragma unroll
  for (int k = 0; k < kTileRun; ++k)
    if (put[k])
      *reinterpret_cast<float2*>(&rec[r[k]].z) = make_float2(ri[k].z + own[k].x, ri[k].w + own[k].y);
  const int frow = cnt > 0 && r0 != rl ? r0 : -1;
  const int cur = rl;
  // the last run of every lane: segmented inclusive scan over the lanes
  const int key = cnt > 0 ? cur : kTileNone;
  const int first = cnt > 0 ? (frow >= 0 ? frow : cur) : kTileNone;
  float sx = cx, sy = cy;
  seg_step<kDppRowShr | 1, 0xF>(key, sx, sy);
  seg_step<kDppRowShr | 2, 0xF>(key, sx, sy);
  seg_step<kDppRowShr | 4, 0xF>(key, sx, sy);
  seg_step<kDppRowShr | 8, 0xF>(key, sx, sy);
  seg_step<kDppRowBcast15, 0xA>(key, sx, sy);
  seg_step<kDppRowBcast31, 0xC>(key, sx, sy);
  if (key == cr.row) {  // lanes continuing the row carried from the previous pass
    sx += cr.x;
    sy += cr.y;
  }
  int pk = dpp_i<kDppWaveShr1, 0xF>(kTileNone - 1, key);
  float px = dpp_f<kDppWaveShr1, 0xF>(0.f, sx), py = dpp_f<kDppWaveShr1, 0xF>(0.f, sy);
  if (lane == 0) {
    pk = cr.row;
    px = cr.x;
    py = cr.y;
    if (cr.row >= 0 && first != cr.row) flush(cr.row, cr.x, cr.y, head, wv, rec, hrow, hval);
  }
  if (frow >= 0) {  // a lane with several runs: its first run ends here
    float tx = fx, ty = fy;
    if (first == pk) {
      tx += px;
      ty += py;
    }
    flush(frow, tx, ty, head, wv, rec, hrow, hval);
  }
  int nf = dpp_i<kDppWaveShl1, 0xF>(kTileNone, first);
  const float lx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sx), kWave - 1));
  const float ly = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sy), kWave - 1));
  const int lk = __builtin_amdgcn_readlane(key, kWave - 1);
  if (lane == kWave - 1) nf = more ? -2 : kTileNone;  // -2: the next pass decides
  if (cnt > 0 && nf != key && nf != -2) flush(key, sx, sy, head, wv, rec, hrow, hval);
  if (more) {
    cr.row = lk;
    cr.x = lx;
    cr.y = ly;
  } else {
    cr.row = -1;
  }
}

__global__ __launch_bounds__(kTileThreads) void k_attract_tiled(TileArgs a) {
  constexpr int PRE = kTileCols / kTileThreads;
  __shared__ float2 win[kTileCols];
  __shared__ float4 rec[kTileMaxRows];  // per slot: x_i and the row's attraction sum
  __shared__ int hrow[kTileWaves];
  __shared__ float2 hval[kTileWaves];
  __shared__ int bst[kTileMaxNC + 1];
  const int t = a.order[blockIdx.x], tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  const int R = a.R, n = a.n;
  const int b0 = a.boff[t], NC = a.boff[t + 1] - b0;  // the tile's windows
  const int xw = a.wlo[t] * kTileCols;                 // first vertex of its first window
  // the tile's block starts: read once, so no window waits on a load of them
  static_assert(kTileMaxNC < kTileThreads, "one block start per thread");
  if (tid <= NC) bst[tid] = a.bstart[(size_t)b0 + tid];
  // the tile's rows and the first window: every load issued before any is used
  {
    int iv[kTileRowsPerThread];
    float2 xv[kTileRowsPerThread], wv0[PRE];
    tile_row_ids(a, t, tid, iv);
#pragma unroll
    for (int q = 0; q < kTileRowsPerThread; ++q) xv[q] = a.X[max(iv[q], 0)];
#pragma unroll
    for (int q = 0; q < PRE; ++q) wv0[q] = a.X[min(xw + q * kTileThreads + tid, n - 1)];
#pragma unroll
    for (int q = 0; q < kTileRowsPerThread; ++q) {
      const int s = q * kTileThreads + tid;
      if (s < R) {
        rec[s] = iv[q] >= 0 ? make_float4(xv[q].x, xv[q].y, 0.f, 0.f) : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
#pragma unroll
    for (int q = 0; q < PRE; ++q) win[q * kTileThreads + tid] = wv0[q];
  }
  if (tid < kTileWaves) hrow[tid] = -1;
  __syncthreads();

  Piece pc = piece_of(a, bst, 0, wv);
  int head = piece_head(pc);
  int s0, cnt;
  run_of(pc.p0, pc.p1, lane, s0, cnt);
  uint2 ec[kTileRun];
#pragma unroll
  for (int k = 0; k < kTileRun; ++k) ec[k] = a.ent[min(s0 + k, a.last)];

  for (int c = 0; c < NC; ++c) {
    const bool has_next = c + 1 < NC;
    const int cn = has_next ? c + 1 : c;  // the last window fetches itself again, unused
    // the next window and the next piece's first run are in flight during this
    // one; the loads are unconditional (clamped indices) so none of them is
    // waited for before it is needed
    float2 pre[PRE];
#pragma unroll
    for (int q = 0; q < PRE; ++q)
      pre[q] = a.X[min(xw + cn * kTileCols + q * kTileThreads + tid, n - 1)];
    const Piece pn = piece_of(a, bst, cn, wv);
    int ns0, ncnt;
    run_of(pn.p0, pn.p1, lane, ns0, ncnt);
    uint2 en[kTileRun];
#pragma unroll
    for (int k = 0; k < kTileRun; ++k) en[k] = a.ent[min(ns0 + k, a.last)];
    Carry cr{-1, 0.f, 0.f};
    if (pc.p0 < pc.p1) {
      // a piece longer than one pass: the entries of each further pass are
      // loaded before the pass ahead of it runs
      constexpr int kPass = kWave * kTileRun;
      uint2 e2[kTileRun];
      int c1 = 0;
      const bool two = pc.p0 + kPass < pc.p1;
      if (two) {
        int s1;
        run_of(pc.p0 + kPass, pc.p1, lane, s1, c1);
#pragma unroll
        for (int k = 0; k < kTileRun; ++k) e2[k] = a.ent[min(s1 + k, a.last)];
      }
      tile_pass(ec, cnt, two, lane, wv, head, win, rec, hrow, hval, cr);
      for (int base = pc.p0 + kPass; base < pc.p1; base += kPass) {
        uint2 cur[kTileRun];
#pragma unroll
        for (int k = 0; k < kTileRun; ++k) cur[k] = e2[k];
        const int cc = c1;
        const bool more = base + kPass < pc.p1;
        if (more) {
          int s1;
          run_of(base + kPass, pc.p1, lane, s1, c1);
#pragma unroll
          for (int k = 0; k < kTileRun; ++k) e2[k] = a.ent[min(s1 + k, a.last)];
        }
        tile_pass(cur, cc, more, lane, wv, head, win, rec, hrow, hval, cr);
      }
    }
    __syncthreads();
    if (wv == 0) {
      // parked partial sums of rows that span pieces, joined per row in wave order
      // (the 16 slots sit in the first row of 16 lanes: row shifts suffice)
      static_assert(kTileWaves == 16, "one DPP row of parking slots");
      const int r = lane < kTileWaves ? hrow[lane] : -1;
      float2 v = make_float2(0.f, 0.f);
      if (r >= 0) v = hval[lane];
      // slots of no row hold -1 and add zeros among themselves
      seg_step<kDppRowShr | 1, 0xF>(r, v.x, v.y);
      seg_step<kDppRowShr | 2, 0xF>(r, v.x, v.y);
      seg_step<kDppRowShr | 4, 0xF>(r, v.x, v.y);
      seg_step<kDppRowShr | 8, 0xF>(r, v.x, v.y);
      int nr = dpp_i<kDppRowShl1, 0xF>(-2, r);
      if (lane == kTileWaves - 1) nr = -2;
      if (lane < kTileWaves && r >= 0 && nr != r) {
        float2* q = reinterpret_cast<float2*>(&rec[r].z);
        *q = make_float2(q->x + v.x, q->y + v.y);
      }
      if (lane < kTileWaves) hrow[lane] = -1;
    }
    if (has_next) {
#pragma unroll
      for (int q = 0; q < PRE; ++q) win[q * kTileThreads + tid] = pre[q];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTileRun; ++k) ec[k] = en[k];
    pc = pn;
    head = piece_head(pn);  // the probes have landed by now
    cnt = ncnt;
  }

  // assembly of the tile's rows (loads batched as at the start)
  int iv[kTileRowsPerThread];
  float4 rv[kTileRowsPerThread];
  tile_row_ids(a, t, tid, iv);
#pragma unroll
  for (int q = 0; q < kTileRowsPerThread; ++q) rv[q] = a.rep_ent[max(iv[q], 0)];
  const int g = a.tgraph[t];
  const double Z = a.zg[g];
  const float inv_z = Z > 0.0 ? (float)(1.0 / Z) : 0.0f;
  const float cn = a.lc * a.gi[g].inv_n, rn = a.lr * a.gi[g].inv_n2;
#pragma unroll
  for (int q = 0; q < kTileRowsPerThread; ++q) {
    const int s = q * kTileThreads + tid, i = iv[q];
    if (i < 0) continue;
    const float4 rs = rec[s];
    const float2 f = make_float2(rs.z, rs.w), xi = make_float2(rs.x, rs.y);
    const float4 re = rv[q];
    const float2 rp = make_float2(re.x, re.y), en = make_float2(re.z, re.w);
    float2 o;
    o.x = a.lkl4 * (f.x - rp.x * inv_z) + cn * xi.x - rn * en.x;
    o.y = a.lkl4 * (f.y - rp.y * inv_z) + cn * xi.y - rn * en.y;
    a.Gout[i] = o;
    if (a.Fattr) a.Fattr[i] = f;
  }
}

hipError_t launch_attract_tiled(Problem& P, const float2* X, const tsnet_params& prm, float2* G,
                                float2* F_attr, hipStream_t s) {
  TileArgs a;
  a.X = X;
  a.n = P.n;
  a.R = P.tile_R;
  a.last = P.nnz > 0 ? (int)(P.nnz - 1) : 0;
  a.tile_rows = P.tile_rows;
  a.wlo = P.tile_wlo;
  a.boff = P.tile_boff;
  a.tgraph = P.tile_graph;
  a.order = P.tile_order;
  a.bstart = P.tile_bstart;
  a.ent = P.tile_ent;
  a.gi = P.ginfo;
  a.zg = P.zg;
  a.rep_ent = P.rep_ent;
  a.lkl4 = (float)(4.0 * prm.lambda_kl);
  a.lc = (float)prm.lambda_c;
  a.lr = (float)prm.lambda_r;
  a.Gout = G;
  a.Fattr = F_attr;
  hipLaunchKernelGGL(k_attract_tiled, dim3(P.tile_T), dim3(kTileThreads), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Layout construction (once per problem).

// keys[e] = (block << kTileSlotBits) | slot of e's row; vals[e] = e.
__global__ __launch_bounds__(256) void k_tile_keys(const int64_t* __restrict__ rowptr,
                                                   const int* __restrict__ col,
                                                   const int* __restrict__ tslot, int n, int R,
                                                   const int* __restrict__ wlo,
                                                   const int* __restrict__ boff, unsigned* keys,
                                                   unsigned* vals) {
  const int lane = lane_id();
  for (int i = blockIdx.x * 4 + wave_id(); i < n; i += gridDim.x * 4) {
    const int ts = tslot[i];
    const unsigned tile = (unsigned)(ts / R), slot = (unsigned)(ts % R);
    const unsigned bt = (unsigned)boff[tile], wt = (unsigned)wlo[tile];
    for (int64_t e = rowptr[i] + lane; e < rowptr[i + 1]; e += kWave) {
      const unsigned b = bt + ((unsigned)col[e] >> kTileColBits) - wt;
      keys[e] = (b << kTileSlotBits) | slot;
      vals[e] = (unsigned)e;
    }
  }
}

__global__ __launch_bounds__(256) void k_tile_fill(const unsigned* __restrict__ keys,
                                                   const unsigned* __restrict__ vals,
                                                   const int* __restrict__ col,
                                                   const float* __restrict__ val, int nnz,
                                                   uint2* ent) {
  for (int p = blockIdx.x * 256 + threadIdx.x; p < nnz; p += gridDim.x * 256) {
    const unsigned e = vals[p];
    const unsigned slot = keys[p] & ((1u << kTileSlotBits) - 1u);
    ent[p] = make_uint2((slot << kTileColBits) | ((unsigned)col[e] & (kTileCols - 1)),
                        __float_as_uint(val[e]));
  }
}

// bstart[b] = first sorted position whose block is >= b, for b in [0, nb].
__global__ __launch_bounds__(256) void k_tile_bounds(const unsigned* __restrict__ keys, int nnz,
                                                     int nb, int* bstart) {
  for (int b = blockIdx.x * 256 + threadIdx.x; b <= nb; b += gridDim.x * 256) {
    int lo = 0, hi = nnz;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((keys[mid] >> kTileSlotBits) < (unsigned)b) lo = mid + 1; else hi = mid;
    }
    bstart[b] = lo;
  }
}

// Row tiles of every graph: at least one per kTileMaxRows rows, and about
// kTileMinTiles in all over the batch (in proportion to the graphs' sizes),
// never more than the graph's rows. Each tile of graph g spans the column
// windows from the one holding g's first vertex to the one holding its last.
struct TilePlan {
  int T = 0, R = 1;
  int64_t nb = 0;
  std::vector<int> first;  // [G + 1] first tile of each graph
  std::vector<int> nw;     // [G] windows of each graph's tiles
  bool ok = false;
};

static TilePlan plan_tiles(const Problem& P) {
  TilePlan tp;
  tp.first.assign(P.G + 1, 0);
  tp.nw.assign(P.G, 0);
  const int64_t n = std::max(P.n, 1);
  for (int g = 0; g < P.G; ++g) {
    const int lo = P.goff[g], ng = P.goff[g + 1] - lo;
    int64_t Tg = 0;
    if (ng > 0) {
      Tg = std::max<int64_t>((ng + kTileMaxRows - 1) / kTileMaxRows,
                             ((int64_t)kTileMinTiles * ng + n - 1) / n);
      Tg = std::min<int64_t>(Tg, ng);
      tp.R = std::max<int>(tp.R, (int)((ng + Tg - 1) / Tg));
      tp.nw[g] = ((lo + ng - 1) >> kTileColBits) - (lo >> kTileColBits) + 1;
      if (tp.nw[g] > kTileMaxNC) return tp;
    }
    tp.first[g + 1] = tp.first[g] + (int)Tg;
    tp.nb += Tg * tp.nw[g];
  }
  tp.T = tp.first[P.G];
  tp.ok = tp.T > 0 && tp.R <= kTileMaxRows && tp.nb < ((int64_t)1 << (32 - kTileSlotBits));
  return tp;
}

bool tiles_supported(const Problem& P) { return plan_tiles(P).ok; }

int build_tiles(Problem& P, hipStream_t s) {
  const int n = P.n;
  const int64_t nnz = P.nnz;
  const TilePlan tp = plan_tiles(P);
  if (!tp.ok) return fail(TSNET_EINVAL, "tiled attraction: a graph spans too many column windows");
  const int T = tp.T, R = tp.R;
  const int nb = (int)tp.nb;
  // rows dealt to each graph's tiles: snake order over decreasing length
  std::vector<int64_t> rp(n + 1);
  TSNET_HIP(hipMemcpyAsync(rp.data(), P.rowptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s));
  TSNET_HIP(hipStreamSynchronize(s));
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::vector<int> tslot(n), rows((size_t)T * R, -1);
  std::vector<int> wlo(T), boff(T + 1), tgraph(T);
  std::vector<int64_t> tnnz(T, 0);  // entries per tile
  for (int g = 0; g < P.G; ++g) {
    const int lo = P.goff[g], hi = P.goff[g + 1];
    const int Tg = tp.first[g + 1] - tp.first[g];
    std::stable_sort(order.begin() + lo, order.begin() + hi, [&](int x, int y) {
      return rp[x + 1] - rp[x] > rp[y + 1] - rp[y];
    });
    for (int q = 0; q < hi - lo; ++q) {
      const int round = q / Tg, idx = q % Tg;
      const int tile = tp.first[g] + ((round & 1) ? Tg - 1 - idx : idx);
      tslot[order[lo + q]] = tile * R + round;
      rows[(size_t)tile * R + round] = order[lo + q];
      tnnz[tile] += rp[order[lo + q] + 1] - rp[order[lo + q]];
    }
    for (int t = tp.first[g]; t < tp.first[g + 1]; ++t) {
      wlo[t] = lo >> kTileColBits;
      tgraph[t] = g;
      boff[t + 1] = boff[t] + tp.nw[g];
    }
  }
  int *rows_d = nullptr, *bstart_d = nullptr, *tslot_d = nullptr;
  // blocks take the tiles largest first, so the last blocks of a launch with
  // more tiles than CUs are the shortest (tiles of one graph are equal)
  std::vector<int> torder(T);
  std::iota(torder.begin(), torder.end(), 0);
  std::stable_sort(torder.begin(), torder.end(), [&](int x, int y) { return tnnz[x] > tnnz[y]; });
  int *wlo_d = nullptr, *boff_d = nullptr, *tgraph_d = nullptr, *torder_d = nullptr;
  uint2* ent_d = nullptr;
  unsigned *keys = nullptr, *vals = nullptr, *kt = nullptr, *vt = nullptr;
  int *hist = nullptr, *tsum = nullptr;
  const int N = (int)nnz;
  const int rtiles = (N + kRadixTile - 1) / kRadixTile;
  const int64_t hist_len = (int64_t)256 * rtiles;
  const int64_t tsum_len = (hist_len + kTileScan - 1) / kTileScan + 8;
  auto release = [](std::initializer_list<void*> ps) {
    for (void* p : ps)
      if (p) (void)hipFree(p);
  };
  auto alloc = [&](auto** p, size_t count, const char* what) -> int {
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(**p));
    if (e != hipSuccess) {
      *p = nullptr;
      return fail(e == hipErrorOutOfMemory ? TSNET_ENOMEM : TSNET_EHIP,
                  std::string("hipMalloc(") + what + "): " + hipGetErrorString(e));
    }
    return TSNET_OK;
  };
  int rc;
  if ((rc = alloc(&rows_d, (size_t)T * R, "tile rows")) ||
      (rc = alloc(&wlo_d, (size_t)T, "tile windows")) ||
      (rc = alloc(&boff_d, (size_t)T + 1, "tile block offsets")) ||
      (rc = alloc(&tgraph_d, (size_t)T, "tile graphs")) ||
      (rc = alloc(&torder_d, (size_t)T, "tile order")) ||
      (rc = alloc(&bstart_d, (size_t)nb + 1, "tile blocks")) ||
      (rc = alloc(&ent_d, (size_t)nnz, "tile entries")) ||
      (rc = alloc(&tslot_d, (size_t)n, "tile slots")) || (rc = alloc(&keys, (size_t)nnz, "keys")) ||
      (rc = alloc(&vals, (size_t)nnz, "vals")) || (rc = alloc(&kt, (size_t)nnz, "keys")) ||
      (rc = alloc(&vt, (size_t)nnz, "vals")) || (rc = alloc(&hist, (size_t)hist_len + 1, "hist")) ||
      (rc = alloc(&tsum, (size_t)tsum_len, "scan"))) {
    release({rows_d, wlo_d, boff_d, tgraph_d, torder_d, bstart_d, ent_d, tslot_d, keys, vals, kt,
             vt, hist, tsum});
    return rc;
  }
  hipError_t e = hipMemcpyAsync(rows_d, rows.data(), sizeof(int) * rows.size(),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(wlo_d, wlo.data(), sizeof(int) * T, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(boff_d, boff.data(), sizeof(int) * (T + 1), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(tgraph_d, tgraph.data(), sizeof(int) * T, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(torder_d, torder.data(), sizeof(int) * T, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(tslot_d, tslot.data(), sizeof(int) * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    int wb = (n + 3) / 4;
    if (wb > 16384) wb = 16384;
    hipLaunchKernelGGL(k_tile_keys, dim3(wb), dim3(256), 0, s, P.rowptr, P.col, tslot_d, n, R,
                       wlo_d, boff_d, keys, vals);
    int bits = kTileSlotBits;
    while (((int64_t)1 << (bits - kTileSlotBits)) <= nb) ++bits;
    e = hipGetLastError();
    if (e == hipSuccess) e = radix_sort(keys, vals, kt, vt, N, bits, hist, tsum, s);
  }
  if (e == hipSuccess) {
    int fb = (int)((nnz + 255) / 256);
    if (fb > 65536) fb = 65536;
    if (fb < 1) fb = 1;
    hipLaunchKernelGGL(k_tile_fill, dim3(fb), dim3(256), 0, s, keys, vals, P.col, P.val, N, ent_d);
    const int bb = (nb + 1 + 255) / 256;
    hipLaunchKernelGGL(k_tile_bounds, dim3(bb < 65536 ? bb : 65536), dim3(256), 0, s, keys, N, nb,
                       bstart_d);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  release({tslot_d, keys, vals, kt, vt, hist, tsum});
  if (e != hipSuccess) {
    release({rows_d, wlo_d, boff_d, tgraph_d, torder_d, bstart_d, ent_d});
    return fail(TSNET_EHIP, std::string("tiled layout: ") + hipGetErrorString(e));
  }
  P.tile_rows = rows_d;
  P.tile_wlo = wlo_d;
  P.tile_boff = boff_d;
  P.tile_graph = tgraph_d;
  P.tile_order = torder_d;
  P.tile_bstart = bstart_d;
  P.tile_ent = ent_d;
  P.tile_T = T;
  P.tile_R = R;
  P.tile_NB = nb;
  return TSNET_OK;
}

}  // namespace tsnet
