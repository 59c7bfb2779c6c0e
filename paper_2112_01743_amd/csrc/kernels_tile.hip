// Batched CPAA kernels: W right-hand sides per tile (an SpMM per term), gfx950.
//
// Tile t stores its vectors vertex-major, Z_t[u*W + j], so gathering
// neighbour v is one coalesced W*4-byte read (W*8 for the FP64 residual).
// A wavefront handles one work item: a group of short rows, 64/W rows at a
// time with one lane per (row, column), or a chunk of a long row whose lane
// groups split the entries and meet through shuffles and an atomic slot
// (the last arriving chunk runs the row's epilogue).  The epilogue is the
// same as the single-vector kernel: D^{-1} scaling, three-term update, FP64
// accumulation and the per-column certificate partial.
#include "device.h"
#include "internal.h"

namespace cpaa {
namespace {

constexpr int kWaves = kWG / 64;
constexpr int kBurst = 8;         // neighbour gathers issued together for a short row
constexpr int kRowsInFlight = 2;  // W = 64: rows whose loads are issued together

// Sum over N(u) of X[v*W + j] for one wavefront work item; epi.row(u, d, j, s, sa)
// is called once per (row, column) by the lane that owns it.
template <typename V, int W, bool ABS, typename Epi>
__device__ __forceinline__ void spmm_item(const WorkItem it, const int* __restrict__ rp,
                                          const int* __restrict__ ci, const V* __restrict__ X,
                                          double* __restrict__ split_part,
                                          int* __restrict__ split_count,
                                          const int* __restrict__ split_nchunks, Epi& epi) {
  constexpr int G = 64 / W;
  const int lane = threadIdx.x & 63;
  const int q = lane / W, j = lane % W;
  if (it.row1 >= 0 && G == 1) {
    // Rows over the whole wavefront (W = 64), several in flight.  The item's row
    // pointers (at most 64 rows) and its first 128 column indices are loaded
    // once, coalesced, and read back with readlane, so the only dependent
    // memory access per row is the burst of neighbour gathers.
    const int nr = it.row1 - it.row0;
    const int cnt = it.nnz1 - it.nnz0;
    const int rpv = lane < nr ? rp[it.row0 + lane] : 0;
    const int civ0 = lane < cnt ? ci[it.nnz0 + lane] : 0;
    const int civ1 = 64 + lane < cnt ? ci[it.nnz0 + 64 + lane] : 0;
    // gathers of row i: up to kBurst neighbours at once (column indices from the
    // item's registers), the rest of a longer row one by one
    auto burst = [&](int beg, int end, V* x) {
#pragma unroll
      for (int u = 0; u < kBurst; ++u) {
        const int k = beg + u - it.nnz0;
        x[u] = V(0);
        if (beg + u < end) {
          int c;
          if (k < 64) c = __builtin_amdgcn_readlane(civ0, k);
          else if (k < 128) c = __builtin_amdgcn_readlane(civ1, k - 64);
          else c = ci[beg + u];
          x[u] = X[(size_t)c * W + j];
        }
      }
    };
    auto finish = [&](int r, int beg, int end, const V* x, const typename Epi::Pre& pre) {
      V s0 = V(0), s1 = V(0), sa = V(0);
#pragma unroll
      for (int u = 0; u < kBurst; u += 2) {
        s0 += x[u];
        s1 += x[u + 1];
        if (ABS) sa += fabs(x[u]) + fabs(x[u + 1]);
      }
      if (end - beg <= kBurst) {
        epi.row(r, end - beg, j, s0 + s1, sa, pre);
        return;
      }
      // rows longer than a burst (up to kTileLongDeg entries, one lane each):
      // the rest is summed in FP64 to keep the rounding independent of degree
      double t0 = static_cast<double>(s0) + static_cast<double>(s1), t1 = 0.0;
      double ta = static_cast<double>(sa);
      int k = beg + kBurst;
      for (; k + 1 < end; k += 2) {
        const V a = X[(size_t)ci[k] * W + j];
        const V b = X[(size_t)ci[k + 1] * W + j];
        t0 += static_cast<double>(a);
        t1 += static_cast<double>(b);
        if (ABS) ta += fabs(static_cast<double>(a)) + fabs(static_cast<double>(b));
      }
      if (k < end) {
        const V a = X[(size_t)ci[k] * W + j];
        t0 += static_cast<double>(a);
        if (ABS) ta += fabs(static_cast<double>(a));
      }
      epi.row(r, end - beg, j, static_cast<V>(t0 + t1), static_cast<V>(ta), pre);
    };
    auto row_end = [&](int i) {
      return i + 1 < nr ? __builtin_amdgcn_readlane(rpv, i + 1) : it.nnz1;
    };
    // kRowsInFlight rows at a time: their operand loads and gathers all go out
    // before the first row's sums are needed
    int i = 0;
    for (; i + kRowsInFlight <= nr; i += kRowsInFlight) {
      int b[kRowsInFlight], e[kRowsInFlight];
      typename Epi::Pre pr[kRowsInFlight];
      V x[kRowsInFlight][kBurst];
#pragma unroll
      for (int f = 0; f < kRowsInFlight; ++f) {
        b[f] = __builtin_amdgcn_readlane(rpv, i + f);
        e[f] = row_end(i + f);
        pr[f] = epi.prefetch(it.row0 + i + f, j);
      }
#pragma unroll
      for (int f = 0; f < kRowsInFlight; ++f) burst(b[f], e[f], x[f]);
#pragma unroll
      for (int f = 0; f < kRowsInFlight; ++f) finish(it.row0 + i + f, b[f], e[f], x[f], pr[f]);
    }
    for (; i < nr; ++i) {
      const int b = __builtin_amdgcn_readlane(rpv, i), e = row_end(i);
      const typename Epi::Pre pr = epi.prefetch(it.row0 + i, j);
      V x[kBurst];
      burst(b, e, x);
      finish(it.row0 + i, b, e, x, pr);
    }
    return;
  }
  if (it.row1 >= 0) {
    // W < 64: 64/W rows at a time, lane (q, j) = (row group, column)
    for (int r = it.row0 + q; r < it.row1; r += G) {
      const int beg = rp[r], end = rp[r + 1];
      // the epilogue's own loads go out first; then up to kBurst neighbour
      // gathers at once, so a short row costs about one memory latency
      const typename Epi::Pre pre = epi.prefetch(r, j);
      V x[kBurst];
#pragma unroll
      for (int u = 0; u < kBurst; ++u)
        x[u] = (beg + u < end) ? X[(size_t)ci[beg + u] * W + j] : V(0);
      V s0 = V(0), s1 = V(0), sa = V(0);
#pragma unroll
      for (int u = 0; u < kBurst; u += 2) {
        s0 += x[u];
        s1 += x[u + 1];
        if (ABS) sa += fabs(x[u]) + fabs(x[u + 1]);
      }
      if (end - beg <= kBurst) {
        epi.row(r, end - beg, j, s0 + s1, sa, pre);
        continue;
      }
      // longer rows (one lane each): the rest is summed in FP64
      double t = static_cast<double>(s0) + static_cast<double>(s1);
      double ta = static_cast<double>(sa);
      for (int k = beg + kBurst; k < end; ++k) {
        const V a = X[(size_t)ci[k] * W + j];
        t += static_cast<double>(a);
        if (ABS) ta += fabs(static_cast<double>(a));
      }
      epi.row(r, end - beg, j, static_cast<V>(t), static_cast<V>(ta), pre);
    }
    return;
  }
  // chunk of a long row: with W = 64 every lane walks the whole chunk, so the
  // chunk and row sums are formed in FP64 (a hub's FP32 sum over thousands of
  // entries would otherwise dominate the recurrence's rounding error)
  double s = 0.0, s2 = 0.0, sa = 0.0;
  int k = it.nnz0 + q;
  for (; k + G < it.nnz1; k += 2 * G) {
    const V a = X[(size_t)ci[k] * W + j];
    const V b = X[(size_t)ci[k + G] * W + j];
    s += static_cast<double>(a);
    s2 += static_cast<double>(b);
    if (ABS) sa += fabs(static_cast<double>(a)) + fabs(static_cast<double>(b));
  }
  if (k < it.nnz1) {
    const V a = X[(size_t)ci[k] * W + j];
    s += static_cast<double>(a);
    if (ABS) sa += fabs(static_cast<double>(a));
  }
  s += s2;
#pragma unroll
  for (int off = W; off < 64; off <<= 1) {
    s += __shfl_xor(s, off);
    if (ABS) sa += __shfl_xor(sa, off);
  }
  const int slot = -(it.row1 + 1);
  double* part = split_part + (size_t)slot * (ABS ? 2 * W : W);
  if (lane < W) {
    atomic_add(&part[j], s);
    if (ABS) atomic_add(&part[W + j], sa);
  }
  atomics_done();
  int prev = 0;
  if (lane == 0) prev = atomicAdd(&split_count[slot], 1);
  prev = __shfl(prev, 0);
  if (prev == split_nchunks[slot] - 1) {
    atomics_done();
    if (lane < W) {
      const double full = __hip_atomic_exchange(&part[j], 0.0, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
      double full_abs = 0.0;
      if (ABS)
        full_abs = __hip_atomic_exchange(&part[W + j], 0.0, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
      epi.row(it.row0, rp[it.row0 + 1] - rp[it.row0], j, static_cast<V>(full),
              static_cast<V>(full_abs), epi.prefetch(it.row0, j));
    }
    if (lane == 0)
      __hip_atomic_exchange(&split_count[slot], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Reduce a per-lane value over the lanes that share column j (lane % W),
// then over the block's wavefronts; the total for column j ends in thread j.
template <int W, typename Op>
__device__ __forceinline__ double column_reduce(double v, double* red /*[kWaves][W]*/, Op op) {
#pragma unroll
  for (int off = W; off < 64; off <<= 1) v = op(v, __shfl_xor(v, off));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane < W) red[w * W + lane] = v;
  __syncthreads();
  double out = 0.0;
  if (threadIdx.x < W) {
    out = red[threadIdx.x];
#pragma unroll
    for (int k = 1; k < kWaves; ++k) out = op(out, red[k * W + threadIdx.x]);
  }
  return out;
}

struct SumOp {
  __device__ double operator()(double a, double b) const { return a + b; }
};
struct MaxOp {
  __device__ double operator()(double a, double b) const { return fmax(a, b); }
};

struct TileTermEpi {
  const float* __restrict__ zc;
  const float* __restrict__ zp;
  float* __restrict__ zn;
  double* __restrict__ acc;
  int W;
  float alpha, gamma_c, gamma;
  AccUpdate au;
  double beta;
  int want_cert;
  double cert;
  struct Pre {
    float zp, zc;
    double acc;
  };
  __device__ __forceinline__ Pre prefetch(int r, int j) const {
    const size_t idx = (size_t)r * W + j;
    // z_{k-1} and acc are read once and written once per launch: streamed with
    // non-temporal accesses so they do not evict the gathered z_k rows
    return {gamma != 0.f || au.a_prev != 0.0 ? __builtin_nontemporal_load(zp + idx) : 0.f,
            (want_cert && beta != 0.0) || au.a_cur != 0.0 || gamma_c != 0.f ? zc[idx] : 0.f,
            au.on ? __builtin_nontemporal_load(acc + idx) : 0.0};
  }
  __device__ __forceinline__ void row(int r, int d, int j, float s, float, const Pre& p) {
    const size_t idx = (size_t)r * W + j;
    float y = alpha * (s / static_cast<float>(d));
    if (gamma_c != 0.f) y -= gamma_c * p.zc;
    if (gamma != 0.f) y -= gamma * p.zp;
    __builtin_nontemporal_store(y, zn + idx);
    if (au.on) {
      // the newest (smallest) term first
      double add = au.a_next * static_cast<double>(y);
      if (au.a_cur != 0.0) add += au.a_cur * static_cast<double>(p.zc);
      if (au.a_prev != 0.0) add += au.a_prev * static_cast<double>(p.zp);
      __builtin_nontemporal_store(p.acc + add, acc + idx);
    }
    if (want_cert)
      cert += static_cast<double>(d) *
              fabs(static_cast<double>(y) - beta * static_cast<double>(p.zc));
  }
};

struct TileTermArgs {
  const int* rp;
  const int* ci;
  const WorkItem* items;
  int n_items;
  int64_t n;
  const float* z_cur;
  const float* z_prev;
  float* z_next;
  double* acc;
  float alpha, gamma_c, gamma;
  AccUpdate au;
  double beta;
  double* cert;        // [kSlots][cols] or null
  int64_t cols;
  const int* done;     // [tiles] or null
  double* split_part;  // [tiles][split slots][W]
  int* split_count;    // [tiles][split slots]
  const int* split_nchunks;
  int n_split;
  int xcd;
};

template <int W>
__global__ __launch_bounds__(kWG) void k_term_tile(TileTermArgs a) {
  const int t = blockIdx.y;
  if (a.done != nullptr && a.done[t]) return;
  const int lb = xcd_logical(blockIdx.x, gridDim.x, a.xcd);
  const int item = __builtin_amdgcn_readfirstlane(lb * kWaves + (threadIdx.x >> 6));
  const size_t off = (size_t)t * a.n * W;
  TileTermEpi epi{a.z_cur + off, a.z_prev ? a.z_prev + off : nullptr, a.z_next + off,
                  a.acc + off, W, a.alpha, a.gamma_c, a.gamma, a.au, a.beta, a.cert != nullptr, 0.0};
  if (item < a.n_items)
    spmm_item<float, W, false>(a.items[item], a.rp, a.ci, a.z_cur + off,
                               a.split_part + (size_t)t * a.n_split * W,
                               a.split_count + (size_t)t * a.n_split, a.split_nchunks, epi);
  if (a.cert != nullptr) {
    __shared__ double red[kWaves * W];
    const double s = column_reduce<W>(epi.cert, red, SumOp());
    if (threadIdx.x < W && s != 0.0)
      atomic_add(&a.cert[(size_t)(lb % kSlots) * a.cols + (size_t)t * W + threadIdx.x], s);
  }
}

struct TileResidEpi {
  const double* __restrict__ acc;
  const double* __restrict__ b;
  double* __restrict__ r_out;
  int W;
  double c;
  double f_abs, f_max, f_q, f_mass, f_round, f_bad;
  struct Pre {
    double acc, b;
  };
  __device__ __forceinline__ Pre prefetch(int r, int j) const {
    const size_t idx = (size_t)r * W + j;
    return {acc[idx], b[idx]};
  }
  __device__ __forceinline__ void row(int r, int d, int j, double s, double sa, const Pre& p) {
    const size_t idx = (size_t)r * W + j;
    const double av = p.acc;
    const double dd = static_cast<double>(d);
    const double bb = p.b;
    const double res = bb - dd * av + c * s;
    r_out[idx] = res;
    const double ar = fabs(res);
    if (!isfinite(res)) f_bad += 1.0;
    f_abs += ar;
    f_max = fmax(f_max, ar);
    f_q += res * res / dd;
    f_mass += dd * av;
    f_round += (dd + 3.0) * 0x1p-53 * (fabs(bb) + dd * fabs(av) + c * sa);
  }
};

struct TileResidArgs {
  const int* rp;
  const int* ci;
  const WorkItem* items;
  int n_items;
  int64_t n;
  const double* acc;
  const double* b;
  double* r;
  double c;
  double* stat_slots;   // residual phase: [kSlots][cols][kStat]
  int64_t cols;
  const int* active;    // [tiles] or null
  double* split_part;   // [tiles][split slots][2][W]
  int* split_count;
  const int* split_nchunks;
  int n_split;
  int xcd;
};

template <int W>
__global__ __launch_bounds__(kWG) void k_resid_tile(TileResidArgs a) {
  const int t = blockIdx.y;
  if (a.active != nullptr && !a.active[t]) return;
  const int lb = xcd_logical(blockIdx.x, gridDim.x, a.xcd);
  const int item = __builtin_amdgcn_readfirstlane(lb * kWaves + (threadIdx.x >> 6));
  const size_t off = (size_t)t * a.n * W;
  TileResidEpi epi{a.acc + off, a.b + off, a.r + off, W, a.c, 0, 0, 0, 0, 0, 0};
  if (item < a.n_items)
    spmm_item<double, W, true>(a.items[item], a.rp, a.ci, a.acc + off,
                               a.split_part + (size_t)t * a.n_split * 2 * W,
                               a.split_count + (size_t)t * a.n_split, a.split_nchunks, epi);
  __shared__ double red[kWaves * W];
  const double v0 = column_reduce<W>(epi.f_abs, red, SumOp());
  const double v1 = column_reduce<W>(epi.f_max, red, MaxOp());
  const double v2 = column_reduce<W>(epi.f_q, red, SumOp());
  const double v3 = column_reduce<W>(epi.f_mass, red, SumOp());
  const double v4 = column_reduce<W>(epi.f_round, red, SumOp());
  const double v5 = column_reduce<W>(epi.f_bad, red, SumOp());
  if (threadIdx.x < W) {
    double* o = a.stat_slots + ((size_t)(lb % kSlots) * a.cols + (size_t)t * W + threadIdx.x) * kStat;
    atomic_add(&o[0], v0);
    atomic_max_nonneg(&o[1], v1);
    atomic_add(&o[2], v2);
    atomic_add(&o[3], v3);
    atomic_add(&o[4], v4);
    if (v5 != 0.0) atomic_add(&o[5], v5);
  }
}

// Caller layout (column j at P + j*ldp) <-> tile layout, through LDS.
// Each workgroup handles 64 consecutive vertices of one tile.
//   mode 0: b = scale*p; z0 = b/d; acc (+)= c0h*b/d (series) ; stats on p
//   mode 1: acc = x0/d; stat [1] counts non-finite x0
template <int W>
__global__ __launch_bounds__(kWG) void k_in_tile(int mode, int64_t n, const int* __restrict__ rp,
                                                 const double* __restrict__ P, int64_t ldp, int B,
                                                 double scale, int add, int store_b, int series,
                                                 double c0h, double* __restrict__ b,
                                                 float* __restrict__ z0, double* __restrict__ acc,
                                                 double* __restrict__ stat_slots, int64_t cols) {
  __shared__ double tile[W][65];
  const int t = blockIdx.y;
  const int64_t u0 = (int64_t)blockIdx.x * 64;
  for (int idx = threadIdx.x; idx < 64 * W; idx += kWG) {
    const int jj = idx / 64, i = idx % 64;
    const int64_t u = u0 + i;
    const int col = t * W + jj;
    tile[jj][i] = (col < B && u < n) ? P[(int64_t)col * ldp + u] : 0.0;
  }
  __syncthreads();
  const size_t off = (size_t)t * n * W;
  double f_sum = 0, f_q = 0, f_neg = 0, f_bad = 0;
  for (int idx = threadIdx.x; idx < 64 * W; idx += kWG) {
    const int i = idx / W, jj = idx % W;   // jj == threadIdx.x % W for every idx
    const int64_t u = u0 + i;
    if (u >= n) continue;
    const double p = tile[jj][i];
    const double d = static_cast<double>(rp[u + 1] - rp[u]);
    const size_t e = off + (size_t)u * W + jj;
    if (mode == 0) {
      const double bu = scale * p;
      const double y = bu / d;
      if (store_b) b[e] = bu;
      if (series) {
        z0[e] = static_cast<float>(y);
        acc[e] = add ? acc[e] + c0h * y : c0h * y;
      }
      f_sum += p;
      f_q += bu * y;
      f_neg += (p < 0.0) ? 1.0 : 0.0;
      f_bad += isfinite(p) ? 0.0 : 1.0;
    } else {
      acc[e] = p / d;
      f_bad += isfinite(p) ? 0.0 : 1.0;
    }
  }
  __shared__ double red[kWaves * W];
  const double v0 = column_reduce<W>(f_sum, red, SumOp());
  const double v2 = column_reduce<W>(f_q, red, SumOp());
  const double v4 = column_reduce<W>(f_neg, red, SumOp());
  const double v5 = column_reduce<W>(f_bad, red, SumOp());
  if (threadIdx.x < W && t * W + (int)threadIdx.x < B) {
    double* o = stat_slots + ((size_t)(blockIdx.x % kSlots) * cols + (size_t)t * W + threadIdx.x) * kStat;
    if (mode == 0) {
      atomic_add(&o[0], v0);
      atomic_add(&o[2], v2);
      if (v4 != 0.0) atomic_add(&o[4], v4);
      if (v5 != 0.0) atomic_add(&o[5], v5);
    } else if (v5 != 0.0) {
      atomic_add(&o[1], v5);
    }
  }
}

// X[col*ldx + u] = col_scale[col] * d_u * acc_tile[u][jj]
template <int W>
__global__ __launch_bounds__(kWG) void k_out_tile(int64_t n, const int* __restrict__ rp,
                                                  const double* __restrict__ acc, int B,
                                                  const double* __restrict__ col_scale,
                                                  double* __restrict__ X, int64_t ldx) {
  __shared__ double tile[W][65];
  const int t = blockIdx.y;
  const int64_t u0 = (int64_t)blockIdx.x * 64;
  const size_t off = (size_t)t * n * W;
  for (int idx = threadIdx.x; idx < 64 * W; idx += kWG) {
    const int i = idx / W, jj = idx % W;
    const int64_t u = u0 + i;
    tile[jj][i] = (u < n) ? static_cast<double>(rp[u + 1] - rp[u]) * acc[off + (size_t)u * W + jj]
                          : 0.0;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 64 * W; idx += kWG) {
    const int jj = idx / 64, i = idx % 64;
    const int64_t u = u0 + i;
    const int col = t * W + jj;
    if (col < B && u < n) X[(int64_t)col * ldx + u] = (col_scale ? col_scale[col] : 1.0) * tile[jj][i];
  }
}

// Series start from the plan's residual (tile layout) for active tiles:
// z0 = r/d, acc += c0h r/d.  Columns flagged in `plain` instead restart as a
// plain solve: acc = 0, r = b (used when a warm start is rejected).
template <int W>
__global__ __launch_bounds__(kWG) void k_from_r_tile(int64_t n, const int* __restrict__ rp,
                                                     double* __restrict__ r,
                                                     const double* __restrict__ b,
                                                     float* __restrict__ z0,
                                                     double* __restrict__ acc, double c0h,
                                                     const int* __restrict__ active,
                                                     const int* __restrict__ plain) {
  const int t = blockIdx.y;
  if (active && !active[t]) return;
  const size_t off = (size_t)t * n * W;
  const size_t total = (size_t)n * W;
  for (size_t e = (size_t)blockIdx.x * kWG + threadIdx.x; e < total; e += (size_t)gridDim.x * kWG) {
    const int64_t u = e / W;
    const int jj = e % W;
    const double d = static_cast<double>(rp[u + 1] - rp[u]);
    double rv = r[off + e];
    double a0 = acc[off + e];
    if (plain && plain[t * W + jj]) {
      rv = b[off + e];
      r[off + e] = rv;
      a0 = 0.0;
    }
    const double y = rv / d;
    z0[off + e] = static_cast<float>(y);
    acc[off + e] = a0 + c0h * y;
  }
}

#define CPAA_LAUNCH_W(KERNEL, W, GRID, ST, ...)                                      \
  do {                                                                              \
    switch (W) {                                                                    \
      case 8: hipLaunchKernelGGL(KERNEL<8>, GRID, dim3(kWG), 0, ST, __VA_ARGS__); break;   \
      case 16: hipLaunchKernelGGL(KERNEL<16>, GRID, dim3(kWG), 0, ST, __VA_ARGS__); break; \
      case 32: hipLaunchKernelGGL(KERNEL<32>, GRID, dim3(kWG), 0, ST, __VA_ARGS__); break; \
      default: hipLaunchKernelGGL(KERNEL<64>, GRID, dim3(kWG), 0, ST, __VA_ARGS__); break; \
    }                                                                               \
  } while (0)

int vert_blocks(int64_t n) { return static_cast<int>((n + 63) / 64); }

}  // namespace

hipError_t init_tile(const cpaa_plan_s* pl, Workspace& ws, const double* P, int64_t ldp, int B,
                     double scale, bool add, bool store_b, bool series, hipStream_t st) {
  CPAA_LAUNCH_W(k_in_tile, ws.W, dim3(vert_blocks(pl->n), ws.tiles), st, 0, (int64_t)pl->n,
                             (const int*)pl->d_row_ptr, P, ldp, B, scale, add ? 1 : 0,
                             store_b ? 1 : 0, series ? 1 : 0, series_a0(pl, ws), ws.b, ws.z[0],
                             ws.acc, ws.stat_slots, ws.cols);
  return hipGetLastError();
}

hipError_t load_x0_tile(const cpaa_plan_s* pl, Workspace& ws, const double* X0, int64_t ldx0,
                        int B, hipStream_t st) {
  CPAA_LAUNCH_W(k_in_tile, ws.W, dim3(vert_blocks(pl->n), ws.tiles), st, 1, (int64_t)pl->n,
                             (const int*)pl->d_row_ptr, X0, ldx0, B, 1.0, 0, 0, 0, 0.0, ws.b,
                             ws.z[0], ws.acc, ws.stat_slots, ws.cols);
  return hipGetLastError();
}

hipError_t init_tile_from_r(const cpaa_plan_s* pl, Workspace& ws, const int* active,
                            const int* plain, hipStream_t st) {
  const size_t total = (size_t)pl->n * ws.W;
  int g = static_cast<int>(std::min<size_t>((total + kWG - 1) / kWG, 8192));
  CPAA_LAUNCH_W(k_from_r_tile, ws.W, dim3(g, ws.tiles), st, (int64_t)pl->n,
                                 (const int*)pl->d_row_ptr, ws.r, (const double*)ws.b, ws.z[0],
                                 ws.acc, series_a0(pl, ws), active, plain);
  return hipGetLastError();
}

hipError_t term_tile(const cpaa_plan_s* pl, Workspace& ws, int cur, int prev, int next, bool first,
                     const AccUpdate& au, double* cert_slot, const int* done, hipStream_t st) {
  const TermShape sh = term_shape(pl, ws, first);
  TileTermArgs a;
  a.rp = pl->d_row_ptr;
  a.ci = pl->d_col_idx;
  a.items = pl->d_titems;
  a.n_items = pl->n_titems;
  a.n = pl->n;
  a.z_cur = ws.z[cur];
  a.z_prev = first ? (sh.zp_is_cur ? ws.z[cur] : nullptr) : ws.z[prev];
  a.z_next = ws.z[next];
  a.acc = ws.acc;
  a.alpha = sh.alpha;
  a.gamma_c = sh.gamma_c;
  a.gamma = sh.gamma;
  a.au = au;
  a.beta = sh.beta;
  a.cert = cert_slot;
  a.cols = ws.cols;
  a.done = done;
  a.split_part = ws.split_d;
  a.split_count = ws.split_count;
  a.split_nchunks = pl->d_tsplit_nchunks;
  a.n_split = pl->n_tsplit_rows;
  a.xcd = pl->xcd_remap_tile;
  const int blocks = (pl->n_titems + kWaves - 1) / kWaves;
  CPAA_LAUNCH_W(k_term_tile, ws.W, dim3(blocks, ws.tiles), st, a);
  return hipGetLastError();
}

hipError_t residual_tile(const cpaa_plan_s* pl, Workspace& ws, const int* active, hipStream_t st) {
  TileResidArgs a;
  a.rp = pl->d_row_ptr;
  a.ci = pl->d_col_idx;
  a.items = pl->d_titems;
  a.n_items = pl->n_titems;
  a.n = pl->n;
  a.acc = ws.acc;
  a.b = ws.b;
  a.r = ws.r;
  a.c = pl->c;
  a.stat_slots = ws.stat_slots + (size_t)kSlots * ws.cols * kStat;
  a.cols = ws.cols;
  a.active = active;
  a.split_part = ws.split_d;
  a.split_count = ws.split_count;
  a.split_nchunks = pl->d_tsplit_nchunks;
  a.n_split = pl->n_tsplit_rows;
  a.xcd = pl->xcd_remap_tile;
  const int blocks = (pl->n_titems + kWaves - 1) / kWaves;
  CPAA_LAUNCH_W(k_resid_tile, ws.W, dim3(blocks, ws.tiles), st, a);
  return hipGetLastError();
}

hipError_t finalize_tile(const cpaa_plan_s* pl, Workspace& ws, double* X, int64_t ldx, int B,
                         const double* col_scale, hipStream_t st) {
  CPAA_LAUNCH_W(k_out_tile, ws.W, dim3(vert_blocks(pl->n), ws.tiles), st, (int64_t)pl->n,
                              (const int*)pl->d_row_ptr, (const double*)ws.acc, B, col_scale, X,
                              ldx);
  return hipGetLastError();
}

}  // namespace cpaa
