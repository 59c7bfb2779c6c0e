// Learned warm start: a small message-passing network that predicts a
// personalized PageRank vector x0 from (log degree, one-hot source); CPAA then
// runs on the residual of x0 (cpaa_solve / cpaa_solve_batched with x0).
//
//   H^0 = [log d, 1{u=s}] (n x 2)         M^l = A D^{-1} H^l  (the paper's P)
//   Z^l = H^l W_self^l + M^l W_nbr^l + b^l,  H^{l+1} = relu(Z^l)   (width 64)
//   score = H^L w_out + b_out,  x0 = softmax(score) over the vertices
//   training loss: cross-entropy -sum_u pi_u log x0_u (pi: a CPAA result);
//   reported error: sum_u |x0_u - pi_u|
//
// Precision: weights, activations H and aggregates M are bfloat16 (round to
// nearest even); every product accumulates in FP32.  The dense layers of
// width 64 run on MFMA (v_mfma_f32_16x16x16bf16_1k); layer 0 (two input
// features) and the head use plain FMA.  The backward pass is FP32 (it uses
// the bf16-rounded weights, as the forward did); its weight gradients and
// input gradients of the width-64 layers run on FP32 MFMA
// (v_mfma_f32_16x16x4f32).  Gradients accumulate over the sources of a step
// in FP32, and Adam updates FP32 master weights from which the bf16 copies
// are re-derived.
//
// Layouts (row-major): H, M: n x 64 bf16 (128 B per vertex, one cache line
// per neighbour gather); H^0, M^0: n x 2 bf16; gradients n x 64 FP32.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "device.h"
#include "internal.h"

namespace cpaa {
namespace {

constexpr int kHid = 64;
constexpr int kIn = 2;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return static_cast<uint16_t>((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

// packed parameter offsets
struct Offs {
  int w_self[4], w_nbr[4], b[4], w_out, b_out, total;
};

Offs make_offs(int layers) {
  Offs o;
  int at = 0, fin = kIn;
  for (int l = 0; l < layers; ++l) {
    o.w_self[l] = at;
    at += fin * kHid;
    o.w_nbr[l] = at;
    at += fin * kHid;
    o.b[l] = at;
    at += kHid;
    fin = kHid;
  }
  o.w_out = at;
  at += kHid;
  o.b_out = at;
  at += 1;
  o.total = at;
  return o;
}

__global__ __launch_bounds__(kWG) void k_invdeg(int n, const int* __restrict__ rp,
                                                float* __restrict__ invd) {
  for (int u = blockIdx.x * kWG + threadIdx.x; u < n; u += gridDim.x * kWG)
    invd[u] = 1.0f / static_cast<float>(rp[u + 1] - rp[u]);
}

// wr = bf16-rounded copy of every weight (biases kept), wt[l] = [W_self; W_nbr]^T in bf16
__global__ __launch_bounds__(kWG) void k_derive(int total, const float* __restrict__ params,
                                                float* __restrict__ wr, int layers, Offs o,
                                                uint16_t* wt1, uint16_t* wt2, uint16_t* wt3) {
  for (int i = blockIdx.x * kWG + threadIdx.x; i < total; i += gridDim.x * kWG) {
    bool is_bias = (i == o.b_out);
    for (int l = 0; l < layers; ++l) is_bias = is_bias || (i >= o.b[l] && i < o.b[l] + kHid);
    wr[i] = is_bias ? params[i] : bf2f(f2bf(params[i]));
  }
  uint16_t* wts[3] = {wt1, wt2, wt3};
  for (int l = 1; l < layers; ++l) {
    for (int i = blockIdx.x * kWG + threadIdx.x; i < kHid * 2 * kHid; i += gridDim.x * kWG) {
      const int col = i / (2 * kHid), k = i % (2 * kHid);
      const float w = k < kHid ? params[o.w_self[l] + k * kHid + col]
                               : params[o.w_nbr[l] + (k - kHid) * kHid + col];
      wts[l - 1][i] = f2bf(w);
    }
  }
}

__global__ __launch_bounds__(kWG) void k_features(int n, const int* __restrict__ rp, int source,
                                                  uint16_t* __restrict__ h0) {
  for (int u = blockIdx.x * kWG + threadIdx.x; u < n; u += gridDim.x * kWG) {
    h0[2 * u] = f2bf(logf(static_cast<float>(rp[u + 1] - rp[u])));
    h0[2 * u + 1] = f2bf(u == source ? 1.0f : 0.0f);
  }
}

// Aggregations walk the plan's wavefront work items (groups of short rows, or
// chunks of a long row whose partial sums meet in an FP32 slot; the last
// chunk to arrive finishes the row), so hub rows of power-law graphs are
// spread over many wavefronts.

// M^0 = A D^{-1} H^0 for the two input features: lanes stride over a row's
// neighbours and reduce with shuffles.
__global__ __launch_bounds__(kWG) void k_agg2(const WorkItem* __restrict__ items, int n_items,
                                              const int* __restrict__ rp,
                                              const int* __restrict__ ci,
                                              const float* __restrict__ invd,
                                              const uint16_t* __restrict__ h,
                                              uint16_t* __restrict__ m, float* __restrict__ part,
                                              int* __restrict__ count,
                                              const int* __restrict__ nchunks) {
  const int lane = threadIdx.x & 63;
  const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (item >= n_items) return;
  const WorkItem it = items[item];
  auto row_sum = [&](int beg, int end, float& a0, float& a1) {
    a0 = a1 = 0.f;
    for (int j = beg + lane; j < end; j += 64) {
      const int v = ci[j];
      const float w = invd[v];
      a0 += bf2f(h[2 * v]) * w;
      a1 += bf2f(h[2 * v + 1]) * w;
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
  };
  if (it.row1 >= 0) {
    for (int r = it.row0; r < it.row1; ++r) {
      float a0, a1;
      row_sum(rp[r], rp[r + 1], a0, a1);
      if (lane == 0) {
        m[2 * r] = f2bf(a0);
        m[2 * r + 1] = f2bf(a1);
      }
    }
    return;
  }
  const int slot = -(it.row1 + 1);
  float a0, a1;
  row_sum(it.nnz0, it.nnz1, a0, a1);
  int prev = 0;
  if (lane == 0) {
    atomicAdd(&part[2 * slot], a0);
    atomicAdd(&part[2 * slot + 1], a1);
    atomics_done();
    prev = atomicAdd(&count[slot], 1);
    if (prev == nchunks[slot] - 1) {
      atomics_done();
      const float f0 = __hip_atomic_exchange(&part[2 * slot], 0.f, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
      const float f1 = __hip_atomic_exchange(&part[2 * slot + 1], 0.f, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_exchange(&count[slot], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      m[2 * it.row0] = f2bf(f0);
      m[2 * it.row0 + 1] = f2bf(f1);
    }
  }
}

// 64-feature aggregation over work items, lane = feature.
//   forward  (BWD = false): M[u] = bf16( sum_{v in N(u)} invd[v] * H[v] ),  H bf16
//   backward (BWD = true) : dH[u] += invd[u] * sum_{v in N(u)} dM[v],       dM FP32
template <bool BWD>
__global__ __launch_bounds__(kWG) void k_agg64(const WorkItem* __restrict__ items, int n_items,
                                               const int* __restrict__ rp,
                                               const int* __restrict__ ci,
                                               const float* __restrict__ invd,
                                               const void* __restrict__ xin,
                                               void* __restrict__ out, float* __restrict__ part,
                                               int* __restrict__ count,
                                               const int* __restrict__ nchunks) {
  const int lane = threadIdx.x & 63;
  const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (item >= n_items) return;
  const WorkItem it = items[item];
  const uint16_t* hb = static_cast<const uint16_t*>(xin);
  const float* xf = static_cast<const float*>(xin);
  auto load = [&](int v) -> float {
    return BWD ? xf[(size_t)v * kHid + lane] : bf2f(hb[(size_t)v * kHid + lane]) * invd[v];
  };
  auto finish = [&](int r, float acc) {
    if (BWD)
      static_cast<float*>(out)[(size_t)r * kHid + lane] += invd[r] * acc;
    else
      static_cast<uint16_t*>(out)[(size_t)r * kHid + lane] = f2bf(acc);
  };
  if (it.row1 >= 0) {
    for (int r = it.row0; r < it.row1; ++r) {
      const int beg = rp[r], end = rp[r + 1];
      float a0 = 0.f, a1 = 0.f;
      int j = beg;
      for (; j + 2 <= end; j += 2) {
        a0 += load(ci[j]);
        a1 += load(ci[j + 1]);
      }
      if (j < end) a0 += load(ci[j]);
      finish(r, a0 + a1);
    }
    return;
  }
  const int slot = -(it.row1 + 1);
  float a0 = 0.f, a1 = 0.f;
  int j = it.nnz0;
  for (; j + 2 <= it.nnz1; j += 2) {
    a0 += load(ci[j]);
    a1 += load(ci[j + 1]);
  }
  if (j < it.nnz1) a0 += load(ci[j]);
  atomicAdd(&part[(size_t)slot * kHid + lane], a0 + a1);
  atomics_done();
  int prev = 0;
  if (lane == 0) prev = atomicAdd(&count[slot], 1);
  prev = __shfl(prev, 0);
  if (prev == nchunks[slot] - 1) {
    atomics_done();
    const float full = __hip_atomic_exchange(&part[(size_t)slot * kHid + lane], 0.f,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    finish(it.row0, full);
    if (lane == 0)
      __hip_atomic_exchange(&count[slot], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// layer 0 dense part (K = 2 + 2): wavefront per vertex, lane = output column
__global__ __launch_bounds__(kWG) void k_dense0(int n, const uint16_t* __restrict__ h0,
                                                const uint16_t* __restrict__ m0,
                                                const float* __restrict__ wr, Offs o,
                                                uint16_t* __restrict__ h1) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * kWG + threadIdx.x) >> 6;
  const int nwaves = (gridDim.x * kWG) >> 6;
  const float ws0 = wr[o.w_self[0] + lane], ws1 = wr[o.w_self[0] + kHid + lane];
  const float wn0 = wr[o.w_nbr[0] + lane], wn1 = wr[o.w_nbr[0] + kHid + lane];
  const float bb = wr[o.b[0] + lane];
  for (int u = wave; u < n; u += nwaves) {
    const float z = bf2f(h0[2 * u]) * ws0 + bf2f(h0[2 * u + 1]) * ws1 + bf2f(m0[2 * u]) * wn0 +
                    bf2f(m0[2 * u + 1]) * wn1 + bb;
    h1[(size_t)u * kHid + lane] = f2bf(fmaxf(z, 0.f));
  }
}

// Dense layer of width 64 on MFMA: Z = [H | M] (n x 128) * [W_self; W_nbr] (128 x 64) + b,
// H' = relu(Z) in bf16.  Each wavefront computes 16 rows x 64 columns with
// v_mfma_f32_16x16x16bf16_1k: lane l supplies A[l%16][4(l/16)..+3] and
// B[4(l/16)..+3][l%16], and receives D[4(l/16)+i][l%16].
__global__ __launch_bounds__(kWG) void k_dense_mfma(int n, const uint16_t* __restrict__ h,
                                                    const uint16_t* __restrict__ m,
                                                    const uint16_t* __restrict__ wt,
                                                    const float* __restrict__ bias,
                                                    uint16_t* __restrict__ hout) {
  __shared__ __attribute__((aligned(16))) uint16_t swt[kHid * 2 * kHid];   // [col][k], k < 128
  __shared__ float sb[kHid];
  for (int i = threadIdx.x; i < kHid * 2 * kHid; i += kWG) swt[i] = wt[i];
  if (threadIdx.x < kHid) sb[threadIdx.x] = bias[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  for (int base = (blockIdx.x * 4 + w) * 16; base < n; base += gridDim.x * 64) {
    floatx4 acc[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int row = base + r16;
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      bf16x4 a = bf16x4{0, 0, 0, 0};
      if (row < n) {
        const uint16_t* src = (ks < 4 ? h : m) + (size_t)row * kHid + (ks & 3) * 16 + kq * 4;
        const uint2 raw = *reinterpret_cast<const uint2*>(src);
        a = __builtin_bit_cast(bf16x4, raw);
      }
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const uint16_t* bsrc = swt + (ct * 16 + r16) * (2 * kHid) + ks * 16 + kq * 4;
        const uint2 rawb = *reinterpret_cast<const uint2*>(bsrc);
        const bf16x4 b = __builtin_bit_cast(bf16x4, rawb);
        acc[ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[ct], 0, 0, 0);
      }
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int col = ct * 16 + r16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = base + kq * 4 + i;
        if (r < n) hout[(size_t)r * kHid + col] = f2bf(fmaxf(acc[ct][i] + sb[col], 0.f));
      }
    }
  }
}

// order-preserving map of a float onto an unsigned key (for an atomic max)
__device__ __forceinline__ unsigned int fkey(float f) {
  const unsigned int b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float key2f(unsigned int k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// score (thread per vertex) and its maximum
__global__ __launch_bounds__(kWG) void k_head(int n, const uint16_t* __restrict__ h,
                                              const float* __restrict__ wr, Offs o,
                                              float* __restrict__ s_out,
                                              unsigned int* __restrict__ smax) {
  __shared__ float sw[kHid];
  if (threadIdx.x < kHid) sw[threadIdx.x] = wr[o.w_out + threadIdx.x];
  __syncthreads();
  const float b_out = wr[o.b_out];
  float mx = -INFINITY;
  for (int u = blockIdx.x * kWG + threadIdx.x; u < n; u += gridDim.x * kWG) {
    const uint4* row = reinterpret_cast<const uint4*>(h + (size_t)u * kHid);
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const uint4 v = row[q];
      const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        s += bf2f(static_cast<uint16_t>(wv[e] & 0xffffu)) * sw[q * 8 + 2 * e];
        s += bf2f(static_cast<uint16_t>(wv[e] >> 16)) * sw[q * 8 + 2 * e + 1];
      }
    }
    s += b_out;
    s_out[u] = s;
    mx = fmaxf(mx, s);
  }
  mx = static_cast<float>(block_max256(static_cast<double>(mx)));
  if (threadIdx.x == 0) atomicMax(smax, fkey(mx));
}

// y = exp(score - max score) and the FP64 sum of y
__global__ __launch_bounds__(kWG) void k_softmax_sum(int n, const float* __restrict__ s,
                                                     const unsigned int* __restrict__ smax,
                                                     float* __restrict__ y,
                                                     double* __restrict__ red) {
  const float mx = key2f(*smax);
  double part = 0.0;
  for (int u = blockIdx.x * kWG + threadIdx.x; u < n; u += gridDim.x * kWG) {
    const float v = expf(s[u] - mx);
    y[u] = v;
    part += v;
  }
  const double tot = block_sum256(part);
  if (threadIdx.x == 0) atomic_add(&red[0], tot);
}

__global__ __launch_bounds__(kWG) void k_normalize(int n, const float* __restrict__ y,
                                                   const double* __restrict__ red,
                                                   double* __restrict__ x0) {
  const double inv = 1.0 / red[0];
  for (int u = blockIdx.x * kWG + threadIdx.x; u < n; u += gridDim.x * kWG)
    x0[u] = static_cast<double>(y[u]) * inv;
}

// red[1] += sum |x0 - pi| (reported error), red[2] += sum pi
__global__ __launch_bounds__(kWG) void k_loss(int n, const double* __restrict__ x0,
                                              const double* __restrict__ pi,
                                              double* __restrict__ red) {
  double l1 = 0.0, ps = 0.0;
  for (int u = blockIdx.x * kWG + threadIdx.x; u < n; u += gridDim.x * kWG) {
    l1 += fabs(x0[u] - pi[u]);
    ps += pi[u];
  }
  l1 = block_sum256(l1);
  ps = block_sum256(ps);
  if (threadIdx.x == 0) {
    atomic_add(&red[1], l1);
    atomic_add(&red[2], ps);
  }
}

// gs = d loss / d score; db_out += sum gs
__global__ __launch_bounds__(kWG) void k_gscore(int n, const double* __restrict__ x0,
                                                const double* __restrict__ pi,
                                                const float* __restrict__ s,
                                                const double* __restrict__ red, float gscale,
                                                float* __restrict__ gs, float* __restrict__ grad,
                                                Offs o) {
  const double psum = red[2];
  double part = 0.0;
  for (int u = blockIdx.x * kWG + threadIdx.x; u < n; u += gridDim.x * kWG) {
    // d(-sum pi log softmax(s)) / d s_u = x0_u sum(pi) - pi_u
    const float g = static_cast<float>(x0[u] * psum - pi[u]) * gscale;
    gs[u] = g;
    part += g;
  }
  part = block_sum256(part);
  if (threadIdx.x == 0) atomicAdd(&grad[o.b_out], static_cast<float>(part));
}

// dw_out[j] += sum_u gs_u H^L[u][j]: wavefront per chunk of rows, lane = feature
__global__ __launch_bounds__(kWG) void k_wout_grad(int n, const float* __restrict__ gs,
                                                   const uint16_t* __restrict__ h,
                                                   float* __restrict__ grad, Offs o, int chunk) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * kWG + threadIdx.x) >> 6;
  const int r0 = wave * chunk;
  if (r0 >= n) return;
  const int r1 = min(n, r0 + chunk);
  float acc = 0.f;
  for (int u = r0; u < r1; ++u) acc += gs[u] * bf2f(h[(size_t)u * kHid + lane]);
  atomicAdd(&grad[o.w_out + lane], acc);
}

// dZ = upstream * 1{H^{l+1} > 0}; upstream is gs (x) w_out for the last layer,
// else dH (FP32).  Wavefront per vertex, lane = column.
__global__ __launch_bounds__(kWG) void k_dz(int n, const uint16_t* __restrict__ hout,
                                            const float* __restrict__ gs,
                                            const float* __restrict__ wr, Offs o,
                                            const float* __restrict__ dh, float* __restrict__ dz) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * kWG + threadIdx.x) >> 6;
  const int nwaves = (gridDim.x * kWG) >> 6;
  const float wo = wr[o.w_out + lane];
  for (int u = wave; u < n; u += nwaves) {
    const size_t e = (size_t)u * kHid + lane;
    const float up = dh ? dh[e] : gs[u] * wo;
    dz[e] = bf2f(hout[e]) > 0.f ? up : 0.f;
  }
}

// dW_self += X^T dZ, dW_nbr += M^T dZ, db += colsum dZ for 64-wide inputs, on
// MFMA (v_mfma_f32_16x16x4f32: FP32 operands, FP32 accumulation, so the
// backward pass keeps its FP32 precision).  Per group of 4
// rows, lane l takes row r0 + l/16 and features 4(l%16)..+3 of X, M and dZ (8,
// 8 and 16 contiguous bytes); tile (t, u) of the 64 x 64 result then holds
// W[4m + t][4c + u] at lane (c = l%16, m = 4(l/16) + i, accumulator i).  Each
// wavefront sums its rows into registers; the workgroup adds its wavefronts'
// sums in LDS in wavefront order and writes one partial [W_self | W_nbr | b]
// (kWgradPart floats) to `part`; k_wgrad_reduce adds the partials in a fixed
// order (no atomics: the same bits on every run).
constexpr int kWgradPart = 2 * kHid * kHid + kHid;
constexpr int kWgradBlocks = 256;   // workgroups of the MFMA weight-gradient pass (at most)
__global__ __launch_bounds__(kWG) void k_wgrad64_mfma(int n, const uint16_t* __restrict__ x,
                                                      const uint16_t* __restrict__ m,
                                                      const float* __restrict__ dz,
                                                      float* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * kWG + threadIdx.x) >> 6;
  const int nwaves = (gridDim.x * kWG) >> 6;
  const int rl = lane >> 4, c = lane & 15;
  floatx4 as[4][4], an[4][4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int u = 0; u < 4; ++u) as[t][u] = an[t][u] = floatx4{0.f, 0.f, 0.f, 0.f};
  float bs[4] = {0.f, 0.f, 0.f, 0.f};
  for (int g = wave; g * 4 < n; g += nwaves) {
    const int r = g * 4 + rl;
    uint2 xr = make_uint2(0u, 0u), mr = make_uint2(0u, 0u);
    float4 zr = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r < n) {
      xr = *reinterpret_cast<const uint2*>(x + (size_t)r * kHid + 4 * c);
      mr = *reinterpret_cast<const uint2*>(m + (size_t)r * kHid + 4 * c);
      zr = *reinterpret_cast<const float4*>(dz + (size_t)r * kHid + 4 * c);
    }
    const float xv[4] = {__uint_as_float(xr.x << 16), __uint_as_float(xr.x & 0xffff0000u),
                         __uint_as_float(xr.y << 16), __uint_as_float(xr.y & 0xffff0000u)};
    const float mv[4] = {__uint_as_float(mr.x << 16), __uint_as_float(mr.x & 0xffff0000u),
                         __uint_as_float(mr.y << 16), __uint_as_float(mr.y & 0xffff0000u)};
    const float zv[4] = {zr.x, zr.y, zr.z, zr.w};
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        as[t][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv[t], zv[u], as[t][u], 0, 0, 0);
        an[t][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(mv[t], zv[u], an[t][u], 0, 0, 0);
      }
#pragma unroll
    for (int u = 0; u < 4; ++u) bs[u] += zv[u];
  }
  // bias: the column sums of this lane's rows, then over the four row lanes
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    bs[u] += __shfl_xor(bs[u], 16);
    bs[u] += __shfl_xor(bs[u], 32);
  }
  __shared__ float red[kWgradPart];
  const int w_in = threadIdx.x >> 6;
  for (int w = 0; w < kWG / 64; ++w) {
    if (w_in == w) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int e = (4 * (4 * rl + i) + t) * kHid + 4 * c + u;
            red[e] = (w == 0 ? 0.f : red[e]) + as[t][u][i];
            red[kHid * kHid + e] = (w == 0 ? 0.f : red[kHid * kHid + e]) + an[t][u][i];
          }
      if (rl == 0)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = 2 * kHid * kHid + 4 * c + u;
          red[e] = (w == 0 ? 0.f : red[e]) + bs[u];
        }
    }
    __syncthreads();
  }
  float* __restrict__ out = part + (size_t)blockIdx.x * kWgradPart;
  for (int e = threadIdx.x; e < kWgradPart; e += kWG) out[e] = red[e];
}

// grad[W_self | W_nbr | b] += the sum of the workgroup partials: each block
// takes 64 entries, its four wavefronts sum four fixed ranges of partials in
// order, and the four range sums are added in order
__global__ __launch_bounds__(kWG) void k_wgrad_reduce(int parts, const float* __restrict__ part,
                                                      float* __restrict__ grad, int o_ws,
                                                      int o_wn, int o_b) {
  __shared__ float seg[kWG / 64][64];
  const int e = blockIdx.x * 64 + (threadIdx.x & 63);
  const int w = threadIdx.x >> 6;
  const int per = (parts + kWG / 64 - 1) / (kWG / 64);
  float s = 0.f;
  if (e < kWgradPart)
    for (int q = w * per; q < min(parts, (w + 1) * per); ++q) s += part[(size_t)q * kWgradPart + e];
  seg[w][threadIdx.x & 63] = s;
  __syncthreads();
  if (threadIdx.x < 64 && e < kWgradPart) {
    float t = seg[0][threadIdx.x];
    for (int q = 1; q < kWG / 64; ++q) t += seg[q][threadIdx.x];
    const int dst = e < kHid * kHid ? o_ws + e
                    : e < 2 * kHid * kHid ? o_wn + (e - kHid * kHid)
                                          : o_b + (e - 2 * kHid * kHid);
    grad[dst] += t;
  }
}

// same for the 2-wide input layer
__global__ __launch_bounds__(kWG) void k_wgrad2(int n, const uint16_t* __restrict__ x,
                                                const uint16_t* __restrict__ m,
                                                const float* __restrict__ dz,
                                                float* __restrict__ grad, Offs o, int chunk) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * kWG + threadIdx.x) >> 6;
  const int r0 = wave * chunk;
  if (r0 >= n) return;
  const int r1 = min(n, r0 + chunk);
  float s0 = 0.f, s1 = 0.f, n0 = 0.f, n1 = 0.f, bb = 0.f;
  for (int u = r0; u < r1; ++u) {
    const float zv = dz[(size_t)u * kHid + lane];
    s0 += bf2f(x[2 * u]) * zv;
    s1 += bf2f(x[2 * u + 1]) * zv;
    n0 += bf2f(m[2 * u]) * zv;
    n1 += bf2f(m[2 * u + 1]) * zv;
    bb += zv;
  }
  atomicAdd(&grad[o.w_self[0] + lane], s0);
  atomicAdd(&grad[o.w_self[0] + kHid + lane], s1);
  atomicAdd(&grad[o.w_nbr[0] + lane], n0);
  atomicAdd(&grad[o.w_nbr[0] + kHid + lane], n1);
  atomicAdd(&grad[o.b[0] + lane], bb);
}

// dHd = dZ W_self^T, dM = dZ W_nbr^T (bf16-rounded weights) on MFMA
// (v_mfma_f32_16x16x4f32): each
// wavefront takes 16 rows; K step s covers columns j = 16 kk + s of dZ (kk =
// l/16: lane l reads its row's 16 contiguous floats 16 kk..+15), B[kk][o] =
// W[o][16 kk + s] from LDS.  Lane l receives dH[r0 + 4(l/16) + i][16 t + l%16].
__global__ __launch_bounds__(kWG) void k_dh_mfma(int n, const float* __restrict__ dz,
                                                 const float* __restrict__ wr, int o_ws,
                                                 int o_wn, float* __restrict__ dhd,
                                                 float* __restrict__ dm) {
  __shared__ float ws[kHid][kHid + 1];   // ws[o][j] = W_self[o][j]
  __shared__ float wn[kHid][kHid + 1];
  for (int i = threadIdx.x; i < kHid * kHid; i += kWG) {
    ws[i / kHid][i % kHid] = wr[o_ws + i];
    wn[i / kHid][i % kHid] = wr[o_wn + i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * kWG + threadIdx.x) >> 6;
  const int nwaves = (gridDim.x * kWG) >> 6;
  const int kk = lane >> 4, c = lane & 15;
  for (int r0 = wave * 16; r0 < n; r0 += nwaves * 16) {
    const int r = r0 + c;
    float a[16];
    if (r < n) {
      const float4* src = reinterpret_cast<const float4*>(dz + (size_t)r * kHid + 16 * kk);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 v = src[q];
        a[4 * q] = v.x;
        a[4 * q + 1] = v.y;
        a[4 * q + 2] = v.z;
        a[4 * q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q) a[q] = 0.f;
    }
    floatx4 hs[4], hn[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) hs[t] = hn[t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int sidx = 0; sidx < 16; ++sidx) {
      const int j = 16 * kk + sidx;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        hs[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[sidx], ws[16 * t + c][j], hs[t], 0, 0, 0);
        hn[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[sidx], wn[16 * t + c][j], hn[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = r0 + 4 * kk + i;
        if (rr < n) {
          dhd[(size_t)rr * kHid + 16 * t + c] = hs[t][i];
          dm[(size_t)rr * kHid + 16 * t + c] = hn[t][i];
        }
      }
  }
}

__global__ __launch_bounds__(kWG) void k_adam(int total, float* __restrict__ w,
                                              const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
  for (int i = blockIdx.x * kWG + threadIdx.x; i < total; i += gridDim.x * kWG) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

int grid_rows(int n, int per_block) {
  const int g = (n + per_block - 1) / per_block;
  return std::max(1, std::min(g, 16384));
}

}  // namespace
}  // namespace cpaa

using namespace cpaa;

struct cpaa_model_s {
  cpaa_plan_s* pl = nullptr;
  int layers = 3;
  int n = 0;
  Offs o{};
  int64_t step = 0;
  float* params = nullptr;   // FP32 master
  float* grads = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  float* wr = nullptr;       // bf16-rounded weights (FP32 storage), biases as is
  uint16_t* wt[3] = {nullptr, nullptr, nullptr};
  float* invd = nullptr;
  uint16_t* h0 = nullptr;
  uint16_t* m0 = nullptr;
  uint16_t* h[4] = {nullptr, nullptr, nullptr, nullptr};   // H^1..H^L
  uint16_t* m[4] = {nullptr, nullptr, nullptr, nullptr};   // M^1..M^{L-1}
  float* s = nullptr;
  float* y = nullptr;
  float* gs = nullptr;
  float* dz = nullptr;
  float* dh = nullptr;
  float* dm = nullptr;
  double* red = nullptr;     // [3] per source
  double* x0tmp = nullptr;   // [n]
  double* hred = nullptr;    // pinned [3]
  float* part = nullptr;     // [long-row slots][64] partial sums of split rows
  int* count = nullptr;      // [long-row slots] chunk arrivals
  float* wpart = nullptr;    // [kWgradBlocks][kWgradPart] weight-gradient partials
};

static void model_free(cpaa_model_s* md) {
  if (!md) return;
  void* ptrs[] = {md->params, md->grads, md->adam_m, md->adam_v, md->wr, md->wt[0], md->wt[1],
                  md->wt[2], md->invd, md->h0, md->m0, md->h[0], md->h[1], md->h[2], md->h[3],
                  md->m[0], md->m[1], md->m[2], md->m[3], md->s, md->y, md->gs, md->dz, md->dh,
                  md->dm, md->red, md->x0tmp, md->part, md->count, md->wpart};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (md->hred) (void)hipHostFree(md->hred);
  delete md;
}

static hipError_t derive(cpaa_model_s* md, hipStream_t st) {
  hipLaunchKernelGGL(k_derive, dim3(64), dim3(kWG), 0, st, md->o.total, md->params, md->wr,
                     md->layers, md->o, md->wt[0], md->wt[1], md->wt[2]);
  return hipGetLastError();
}

// forward pass for one source; x0 (n FP64) and the activations stay on device
static hipError_t forward(cpaa_model_s* md, int source, double* x0, hipStream_t st) {
  cpaa_plan_s* pl = md->pl;
  const int n = md->n;
  const int gw = grid_rows(n, 4);      // wavefront-per-vertex kernels: 4 vertices per block pass
  const int ge = grid_rows(n, kWG);
  hipLaunchKernelGGL(k_features, dim3(ge), dim3(kWG), 0, st, n, pl->d_row_ptr, source, md->h0);
  const dim3 gi((pl->n_titems + 3) / 4);
  hipLaunchKernelGGL(k_agg2, gi, dim3(kWG), 0, st, pl->d_titems, pl->n_titems, pl->d_row_ptr,
                     pl->d_col_idx, md->invd, md->h0, md->m0, md->part, md->count,
                     pl->d_tsplit_nchunks);
  hipLaunchKernelGGL(k_dense0, dim3(gw), dim3(kWG), 0, st, n, md->h0, md->m0, md->wr, md->o,
                     md->h[0]);
  for (int l = 1; l < md->layers; ++l) {
    hipLaunchKernelGGL(k_agg64<false>, gi, dim3(kWG), 0, st, pl->d_titems, pl->n_titems,
                       pl->d_row_ptr, pl->d_col_idx, md->invd, (const void*)md->h[l - 1],
                       (void*)md->m[l - 1], md->part, md->count, pl->d_tsplit_nchunks);
    hipLaunchKernelGGL(k_dense_mfma, dim3(grid_rows(n, 64)), dim3(kWG), 0, st, n, md->h[l - 1],
                       md->m[l - 1], md->wt[l - 1], md->params + md->o.b[l], md->h[l]);
  }
  // red[0..2]: softmax sum, loss, sum of targets; red[3]: score maximum key
  hipError_t e = fill_f64(md->red, 0.0, 4, st);
  if (e != hipSuccess) return e;
  unsigned int* smax = reinterpret_cast<unsigned int*>(md->red + 3);
  hipLaunchKernelGGL(k_head, dim3(ge), dim3(kWG), 0, st, n, md->h[md->layers - 1], md->wr, md->o,
                     md->s, smax);
  hipLaunchKernelGGL(k_softmax_sum, dim3(ge), dim3(kWG), 0, st, n, md->s, smax, md->y, md->red);
  hipLaunchKernelGGL(k_normalize, dim3(ge), dim3(kWG), 0, st, n, md->y, md->red, x0);
  return hipGetLastError();
}

// backward pass after forward() for the same source; adds gscale * gradient to md->grads
static hipError_t backward(cpaa_model_s* md, const double* x0, const double* pi, float gscale,
                           hipStream_t st) {
  cpaa_plan_s* pl = md->pl;
  const int n = md->n;
  const int L = md->layers;
  const int gw = grid_rows(n, 4);
  const int ge = grid_rows(n, kWG);
  hipLaunchKernelGGL(k_loss, dim3(ge), dim3(kWG), 0, st, n, x0, pi, md->red);
  hipLaunchKernelGGL(k_gscore, dim3(ge), dim3(kWG), 0, st, n, x0, pi, md->s, md->red, gscale,
                     md->gs, md->grads, md->o);
  const int chunk_w = 256;
  hipLaunchKernelGGL(k_wout_grad, dim3(std::max(1, (n + chunk_w * 4 - 1) / (chunk_w * 4))),
                     dim3(kWG), 0, st, n, md->gs, md->h[L - 1], md->grads, md->o, chunk_w);
  for (int l = L - 1; l >= 0; --l) {
    // dZ^l from upstream (gs w_out for the last layer, dH^{l+1} otherwise)
    hipLaunchKernelGGL(k_dz, dim3(gw), dim3(kWG), 0, st, n, md->h[l], md->gs, md->wr, md->o,
                       l == L - 1 ? nullptr : md->dh, md->dz);
    if (l >= 1) {
      // workgroups of 4 wavefronts, 16 rows per wavefront group step
      const int wg_blocks = std::max(1, std::min(kWgradBlocks, (n + 1023) / 1024));
      hipLaunchKernelGGL(k_wgrad64_mfma, dim3(wg_blocks), dim3(kWG), 0, st, n, md->h[l - 1],
                         md->m[l - 1], md->dz, md->wpart);
      hipLaunchKernelGGL(k_wgrad_reduce, dim3((kWgradPart + 63) / 64), dim3(kWG), 0, st,
                         wg_blocks, md->wpart, md->grads, md->o.w_self[l], md->o.w_nbr[l],
                         md->o.b[l]);
      hipLaunchKernelGGL(k_dh_mfma, dim3(grid_rows(n, 64)), dim3(kWG), 0, st, n, md->dz, md->wr,
                         md->o.w_self[l], md->o.w_nbr[l], md->dh, md->dm);
      hipLaunchKernelGGL(k_agg64<true>, dim3((pl->n_titems + 3) / 4), dim3(kWG), 0, st,
                         pl->d_titems, pl->n_titems, pl->d_row_ptr, pl->d_col_idx, md->invd,
                         (const void*)md->dm, (void*)md->dh, md->part, md->count,
                         pl->d_tsplit_nchunks);
    } else {
      const int chunk = 256;
      hipLaunchKernelGGL(k_wgrad2, dim3(std::max(1, (n + chunk * 4 - 1) / (chunk * 4))),
                         dim3(kWG), 0, st, n, md->h0, md->m0, md->dz, md->grads, md->o, chunk);
    }
  }
  return hipGetLastError();
}

extern "C" {

cpaa_status cpaa_model_create(cpaa_plan_t pl, int32_t layers, int32_t hidden, const float* params,
                              cpaa_model_t* out) {
  set_error("");
  if (!pl || !params || !out) {
    set_error("cpaa_model_create: null argument");
    return CPAA_EINVAL;
  }
  *out = nullptr;
  if (layers < 1 || layers > 4 || hidden != kHid || pl->num_graphs > 1 || pl->directed ||
      pl->n_drop > 0) {
    set_error("the warm-start network supports 1..4 layers of width 64 on a single-graph "
              "undirected plan without dropped vertices");
    return CPAA_EINVAL;
  }
  cpaa_model_s* md = new (std::nothrow) cpaa_model_s();
  if (!md) {
    set_error("host allocation failed");
    return CPAA_ENOMEM;
  }
  md->pl = pl;
  md->layers = layers;
  md->n = pl->n;
  md->o = make_offs(layers);
  const size_t n = pl->n;
  const size_t P = md->o.total;
  bool ok = true;
  auto A = [&](void** p, size_t bytes) {
    if (!ok) return;
    if (hipMalloc(p, std::max<size_t>(bytes, 8)) != hipSuccess) {
      (void)hipGetLastError();
      ok = false;
    }
  };
  A((void**)&md->params, P * 4);
  A((void**)&md->grads, P * 4);
  A((void**)&md->adam_m, P * 4);
  A((void**)&md->adam_v, P * 4);
  A((void**)&md->wr, P * 4);
  for (int l = 1; l < layers; ++l) A((void**)&md->wt[l - 1], kHid * 2 * kHid * 2);
  A((void**)&md->invd, n * 4);
  A((void**)&md->h0, n * kIn * 2);
  A((void**)&md->m0, n * kIn * 2);
  for (int l = 0; l < layers; ++l) A((void**)&md->h[l], n * kHid * 2);
  for (int l = 0; l + 1 < layers; ++l) A((void**)&md->m[l], n * kHid * 2);
  A((void**)&md->s, n * 4);
  A((void**)&md->y, n * 4);
  A((void**)&md->gs, n * 4);
  A((void**)&md->dz, n * kHid * 4);
  A((void**)&md->dh, n * kHid * 4);
  A((void**)&md->dm, n * kHid * 4);
  A((void**)&md->red, 4 * 8);
  A((void**)&md->x0tmp, n * 8);
  const size_t nslots = std::max(pl->n_tsplit_rows, 1);
  A((void**)&md->part, nslots * kHid * 4);
  A((void**)&md->count, nslots * 4);
  A((void**)&md->wpart, (size_t)kWgradBlocks * kWgradPart * 4);
  if (ok && hipHostMalloc((void**)&md->hred, 4 * 8, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    ok = false;
  }
  if (!ok) {
    model_free(md);
    set_error("device allocation for the warm-start network failed");
    return CPAA_ENOMEM;
  }
  if (hipMemcpy(md->params, params, P * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(md->part, 0, nslots * kHid * 4) != hipSuccess ||
      hipMemset(md->count, 0, nslots * 4) != hipSuccess ||
      hipMemset(md->adam_m, 0, P * 4) != hipSuccess || hipMemset(md->adam_v, 0, P * 4) != hipSuccess) {
    model_free(md);
    set_error("upload of the network parameters failed");
    return CPAA_EDEVICE;
  }
  hipLaunchKernelGGL(k_invdeg, dim3(grid_rows(md->n, kWG)), dim3(kWG), 0, nullptr, md->n,
                     pl->d_row_ptr, md->invd);
  if (derive(md, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    model_free(md);
    set_error("network set-up kernels failed");
    return CPAA_EDEVICE;
  }
  *out = md;
  return CPAA_OK;
}

void cpaa_model_destroy(cpaa_model_t md) { model_free(md); }

int32_t cpaa_model_num_params(cpaa_model_t md) { return md ? md->o.total : 0; }

cpaa_status cpaa_model_get_state(cpaa_model_t md, float* params, float* adam_m, float* adam_v,
                                 int64_t* step) {
  if (!md) {
    set_error("null model");
    return CPAA_EINVAL;
  }
  const size_t bytes = (size_t)md->o.total * 4;
  if (params) CPAA_HIP(hipMemcpy(params, md->params, bytes, hipMemcpyDeviceToHost));
  if (adam_m) CPAA_HIP(hipMemcpy(adam_m, md->adam_m, bytes, hipMemcpyDeviceToHost));
  if (adam_v) CPAA_HIP(hipMemcpy(adam_v, md->adam_v, bytes, hipMemcpyDeviceToHost));
  if (step) *step = md->step;
  return CPAA_OK;
}

cpaa_status cpaa_model_set_state(cpaa_model_t md, const float* params, const float* adam_m,
                                 const float* adam_v, int64_t step) {
  if (!md || !params) {
    set_error("null model or parameters");
    return CPAA_EINVAL;
  }
  const size_t bytes = (size_t)md->o.total * 4;
  CPAA_HIP(hipMemcpy(md->params, params, bytes, hipMemcpyHostToDevice));
  if (adam_m) CPAA_HIP(hipMemcpy(md->adam_m, adam_m, bytes, hipMemcpyHostToDevice));
  if (adam_v) CPAA_HIP(hipMemcpy(md->adam_v, adam_v, bytes, hipMemcpyHostToDevice));
  md->step = step;
  CPAA_HIP(derive(md, nullptr));
  CPAA_HIP(hipDeviceSynchronize());
  return CPAA_OK;
}

cpaa_status cpaa_model_predict(cpaa_model_t md, int32_t B, const int32_t* sources, double* X0,
                               int64_t ldx, void* stream) {
  set_error("");
  if (!md || !sources || !X0 || B <= 0 || ldx < md->n) {
    set_error("cpaa_model_predict: bad argument");
    return CPAA_EINVAL;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  for (int j = 0; j < B; ++j) {
    if (sources[j] < 0 || sources[j] >= md->n) {
      set_error("source out of range");
      return CPAA_EINVAL;
    }
  }
  for (int j = 0; j < B; ++j) CPAA_HIP(forward(md, sources[j], X0 + (size_t)j * ldx, st));
  CPAA_HIP(hipStreamSynchronize(st));
  return CPAA_OK;
}

// Forward + backward for B sources against targets (columns of T), gradients
// averaged over the sources.  With lr > 0 an Adam step follows; grads_out
// (host, may be NULL) receives the averaged gradient; loss_out the mean loss.
cpaa_status cpaa_model_train_step(cpaa_model_t md, int32_t B, const int32_t* sources,
                                  const double* T, int64_t ldt, float lr, float* grads_out,
                                  double* loss_out, void* stream) {
  set_error("");
  if (!md || !sources || !T || B <= 0 || ldt < md->n) {
    set_error("cpaa_model_train_step: bad argument");
    return CPAA_EINVAL;
  }
  for (int j = 0; j < B; ++j) {
    if (sources[j] < 0 || sources[j] >= md->n) {
      set_error("source out of range");
      return CPAA_EINVAL;
    }
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  CPAA_HIP(hipMemsetAsync(md->grads, 0, (size_t)md->o.total * 4, st));
  double loss = 0.0;
  for (int j = 0; j < B; ++j) {
    CPAA_HIP(forward(md, sources[j], md->x0tmp, st));
    CPAA_HIP(backward(md, md->x0tmp, T + (size_t)j * ldt, 1.0f / B, st));
    CPAA_HIP(hipMemcpyAsync(md->hred, md->red, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    CPAA_HIP(hipStreamSynchronize(st));
    loss += md->hred[1];
  }
  if (grads_out)
    CPAA_HIP(hipMemcpy(grads_out, md->grads, (size_t)md->o.total * 4, hipMemcpyDeviceToHost));
  if (lr > 0.f) {
    md->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)md->step), c2 = 1.f - std::pow(b2, (float)md->step);
    hipLaunchKernelGGL(k_adam, dim3(64), dim3(kWG), 0, st, md->o.total, md->params, md->grads,
                       md->adam_m, md->adam_v, lr, b1, b2, 1e-8f, c1, c2);
    CPAA_HIP(hipGetLastError());
    CPAA_HIP(derive(md, st));
    CPAA_HIP(hipStreamSynchronize(st));
  }
  if (loss_out) *loss_out = loss / B;
  return CPAA_OK;
}

}  // extern "C"
