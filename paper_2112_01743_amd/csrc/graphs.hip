// Uneven batch of small independent graphs solved in one persistent launch.
//
// The plan holds a block-diagonal graph (graph g owns vertices
// [graph_ptr[g], graph_ptr[g+1])).  Each workgroup repeatedly takes the next
// graph from an atomic queue (graphs ordered by stored entries, largest
// first) and solves it completely on chip:
//   * the graph's Chebyshev vectors live in LDS (FP32, z-space), the FP64
//     accumulator, right-hand side and residual live in registers (a fixed set
//     of rows per thread);
//   * one term is one pass over the graph's entries, stored as packed local
//     (row, column) 16-bit pairs in per-lane runs (see coo_pass): gather z
//     from LDS, sum rows in registers, so every thread gets the same number
//     of entries whatever the degree distribution;
//   * the three-term update, D^{-1} scaling and FP64 accumulation follow in the
//     epilogue, and from the mass-error bound on (eq. 4.1) the workgroup
//     evaluates the in-loop certificate and stops that graph on its own;
//   * the FP64 residual (with its rounding allowance) and, if needed,
//     correction series run in the same workgroup, then D acc is written out.
// Graphs are split into size classes by vertex count; each class is one
// persistent launch with the LDS of its largest graph and its own workgroup
// size (timed per class on the first call when autotuning).  The host captures
// "reset queues -> validate p -> one launch per class" once in a HIP graph per
// (p, x, tol) and replays it.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "device.h"
#include "internal.h"

namespace cpaa {
namespace {

constexpr int kRec = 12;
constexpr int kGraphRunMax = 16;               // longest per-lane run of packed entries
constexpr uint32_t kGraphPad = 0xFFFFFFFFu;    // padding entry (row 0xffff never exists)
// record fields
enum { R_TERMS, R_REF_TERMS, R_REFS, R_BOUND, R_RL1, R_RMAX, R_MASS, R_SCERT, R_PSUM, R_PNEG,
       R_PBAD, R_CERTIFIED };

struct GraphArgs {
  const int* rp;
  const uint32_t* coo;      // (local_row << 16) | local_col, per graph in transposed runs
  const int* coo_off;       // [num_graphs] first packed entry of each graph
  const int* coo_meta;      // [num_graphs] chunks << 6 | run length
  const int* graph_ptr;
  const int* order;
  int num_graphs;
  int max_ng;               // LDS sizing (vertices)
  int* queue;
  const int* abort;
  const double* p;
  double* x;
  double c, s, beta, c0h;
  double tol, target_main, target_ref;
  int k_min, k_cap_max, max_refine, normalize;
  double* rec;              // [num_graphs][kRec]
};

// Sum / max over the workgroup, returned to every thread: wavefront partials
// through LDS, then each wavefront reduces the partials across its lanes (the
// same butterfly in every wavefront, so every thread gets the same bits).
template <int BLOCK>
__device__ __forceinline__ double block_allsum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  return wave_sum(lane < BLOCK / 64 ? red[lane] : 0.0);
}

template <int BLOCK>
__device__ __forceinline__ double block_allmax(double v, double* red) {
  v = wave_max(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  return wave_max(lane < BLOCK / 64 ? red[lane] : 0.0);
}

// y[row] += src[col] over the graph's entries (LDS gathers, LDS atomics).
// One pass y[row] += src[col] (or |src[col]|) over a graph's packed entries.
// The entries of each chunk of 64*rl (row-ordered) entries are stored
// transposed: lane l owns the contiguous run [l*rl, (l+1)*rl) (rl a multiple
// of 4), elements 4q..4q+3 of the run at q*256 + 4l, so each lane reads four
// run elements with one 16-byte load and a wavefront's load covers 1 KB
// contiguously, while a lane sums its rows in a register.  A row that starts and ends inside a run has no other contributor
// (plain LDS store into the zeroed y); the first and last row of a run may be
// shared with neighbouring runs (LDS atomic).  Per-entry LDS atomics, with
// the lanes of a wavefront mostly hitting the same row, cost 4x more.
template <int BLOCK, typename T, bool ABS>
__device__ __forceinline__ void coo_pass(const uint32_t* __restrict__ coo, int nch, int rl,
                                         const T* src, T* y) {
  const int lane = threadIdx.x & 63;
  for (int c = threadIdx.x >> 6; c < nch; c += BLOCK / 64) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4* pc = reinterpret_cast<const u32x4*>(coo + (size_t)c * 64 * rl) + lane;
    uint32_t e[kGraphRunMax];
#pragma unroll
    for (int q = 0; q < kGraphRunMax / 4; ++q) {
      const u32x4 v = 4 * q < rl ? pc[q * 64] : u32x4{kGraphPad, kGraphPad, kGraphPad, kGraphPad};
      e[4 * q] = v.x;
      e[4 * q + 1] = v.y;
      e[4 * q + 2] = v.z;
      e[4 * q + 3] = v.w;
    }
    int row = -1;
    T sum = T(0);
    bool first = true;
#pragma unroll
    for (int i = 0; i < kGraphRunMax; ++i) {
      T vi = e[i] != kGraphPad ? src[e[i] & 0xffffu] : T(0);
      if (ABS) vi = fabs(vi);
      if (e[i] != kGraphPad) {
        const int r = static_cast<int>(e[i] >> 16);
        if (r != row) {
          if (row >= 0) {
            if (first)
              atomicAdd(&y[row], sum);
            else
              y[row] = sum;
            first = false;
          }
          row = r;
          sum = vi;
        } else {
          sum += vi;
        }
      }
    }
    if (row >= 0) atomicAdd(&y[row], sum);
  }
}

template <int BLOCK, int RPT>
__device__ void solve_graph(const GraphArgs& a, int g, unsigned char* lds, double* red,
                            int* bcast) {
  const int t = threadIdx.x;
  const int v0 = a.graph_ptr[g];
  const int ng = a.graph_ptr[g + 1] - v0;
  const uint32_t* coo = a.coo + a.coo_off[g];
  const int nch = a.coo_meta[g] >> 6, rl = a.coo_meta[g] & 63;
  // LDS regions: A = 8*max_ng bytes, B = 8*max_ng bytes
  float* za = reinterpret_cast<float*>(lds);
  float* zb = za + a.max_ng;
  float* yf = reinterpret_cast<float*>(lds + 8 * (size_t)a.max_ng);
  double* ad = reinterpret_cast<double*>(lds);
  double* yd = reinterpret_cast<double*>(lds + 8 * (size_t)a.max_ng);

  double bb[RPT], acc[RPT], rr[RPT];
  float dd[RPT];
  double q = 0.0, vol = 0.0;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int u = t + i * BLOCK;
    bb[i] = acc[i] = rr[i] = 0.0;
    dd[i] = 0.f;
    if (u < ng) {
      const int d = a.rp[v0 + u + 1] - a.rp[v0 + u];
      const double b = (1.0 - a.c) * a.p[v0 + u];
      bb[i] = b;
      dd[i] = static_cast<float>(d);
      q += b * b / d;
      vol += d;
    }
  }
  q = block_allsum<BLOCK>(q, red);
  vol = block_allsum<BLOCK>(vol, red);

  const double tail0 = 2.0 / a.s / (1.0 - a.beta);   // sum_{k>M} c_k = tail0 * beta^{M+1}
  auto apriori = [&](double qq, double target) {
    const double scale = sqrt(vol) * sqrt(fmax(qq, 0.0)) * tail0;
    int M = 0;
    double bp = a.beta;
    while (M < a.k_cap_max && scale * bp > target) {
      ++M;
      bp *= a.beta;
    }
    return M;
  };

  int terms_main = 0, ref_terms = 0, refs = 0;
  double series_cert = -1.0, bound = 0.0, r_l1 = 0.0, r_max = 0.0, mass = 0.0;
  bool first_series = true;
  double qs = q;
  for (;;) {
    // ---- one series on b' (bb for the first, rr for corrections) ----
    const double target = first_series ? a.target_main : a.target_ref;
    const int k_cap = apriori(qs, target);
    const int k_min = first_series ? min(a.k_min, k_cap) : 1;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int u = t + i * BLOCK;
      if (u < ng) {
        const double y0 = (first_series ? bb[i] : rr[i]) / dd[i];
        za[u] = static_cast<float>(y0);
        acc[i] = (first_series ? 0.0 : acc[i]) + a.c0h * y0;
        yf[u] = 0.f;
      }
    }
    __syncthreads();
    int terms = 0;
    double ck = 2.0 * a.c0h;   // c_0
    if (k_cap >= 1) {
      coo_pass<BLOCK, float, false>(coo, nch, rl, za, yf);
      __syncthreads();
      ck *= a.beta;            // c_1
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int u = t + i * BLOCK;
        if (u < ng) {
          const float z1 = yf[u] / dd[i];
          zb[u] = z1;
          acc[i] += ck * static_cast<double>(z1);
          yf[u] = 0.f;
        }
      }
      __syncthreads();
      terms = 1;
    }
    float* cur = zb;
    float* prv = za;
    double bpow = a.beta * a.beta;   // beta^{k+1} for k = 1
    for (int k = 1; k < k_cap; ++k) {
      coo_pass<BLOCK, float, false>(coo, nch, rl, cur, yf);
      __syncthreads();
      ck *= a.beta;            // c_{k+1}
      const bool want = k >= k_min;
      double cert = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int u = t + i * BLOCK;
        if (u < ng) {
          const float zn = 2.f * (yf[u] / dd[i]) - prv[u];
          if (want)
            cert += static_cast<double>(dd[i]) *
                    fabs(static_cast<double>(zn) - a.beta * static_cast<double>(cur[u]));
          prv[u] = zn;
          acc[i] += ck * static_cast<double>(zn);
          yf[u] = 0.f;
        }
      }
      terms = k + 1;
      float* tmp = cur;
      cur = prv;
      prv = tmp;
      bool stop = false;
      if (want) {
        const double cs = block_allsum<BLOCK>(cert, red) * (1.0 + a.s) / a.s * bpow / (1.0 - a.c);
        series_cert = cs;
        stop = cs <= target;
      }
      bpow *= a.beta;
      __syncthreads();
      if (stop) break;
    }
    if (first_series)
      terms_main = terms;
    else
      ref_terms += terms;

    // ---- FP64 residual r = b - (I - cP) x with x = D acc ----
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int u = t + i * BLOCK;
      if (u < ng) {
        ad[u] = acc[i];
        yd[u] = 0.0;
      }
    }
    __syncthreads();
    coo_pass<BLOCK, double, false>(coo, nch, rl, ad, yd);
    __syncthreads();
    double f_abs = 0.0, f_max = 0.0, f_q = 0.0, f_mass = 0.0, f_round = 0.0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int u = t + i * BLOCK;
      if (u < ng) {
        const double d = dd[i];
        const double r = bb[i] - d * acc[i] + a.c * yd[u];
        rr[i] = r;
        f_abs += fabs(r);
        f_max = fmax(f_max, fabs(r));
        f_q += r * r / d;
        f_mass += d * acc[i];
        yd[u] = 0.0;
      }
    }
    __syncthreads();
    coo_pass<BLOCK, double, true>(coo, nch, rl, ad, yd);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int u = t + i * BLOCK;
      if (u < ng) {
        const double d = dd[i];
        f_round += (d + 3.0) * 0x1p-53 * (fabs(bb[i]) + d * fabs(acc[i]) + a.c * yd[u]);
      }
    }
    r_l1 = block_allsum<BLOCK>(f_abs, red);
    r_max = block_allmax<BLOCK>(f_max, red);
    qs = block_allsum<BLOCK>(f_q, red);
    mass = block_allsum<BLOCK>(f_mass, red);
    const double rnd = block_allsum<BLOCK>(f_round, red);
    const double u53 = 0x1p-53;
    bound = (r_l1 * (1.0 + 2.0 * u53 * ng) + rnd) / (1.0 - a.c) + u53 * fabs(mass);
    first_series = false;
    if (bound <= a.tol || !isfinite(bound) || refs >= a.max_refine) break;
    ++refs;
  }
  __syncthreads();
  const double scale = a.normalize ? 1.0 / mass : 1.0;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int u = t + i * BLOCK;
    if (u < ng) a.x[v0 + u] = scale * static_cast<double>(dd[i]) * acc[i];
  }
  if (t == 0) {
    double* r = a.rec + (size_t)g * kRec;
    r[R_TERMS] = terms_main;
    r[R_REF_TERMS] = ref_terms;
    r[R_REFS] = refs;
    r[R_BOUND] = bound;
    r[R_RL1] = r_l1;
    r[R_RMAX] = r_max;
    r[R_MASS] = a.normalize ? 1.0 : mass;
    r[R_SCERT] = series_cert;
    r[R_CERTIFIED] = bound <= a.tol ? 1.0 : 0.0;
  }
  (void)bcast;
}

template <int BLOCK, int RPT>
__global__ __launch_bounds__(BLOCK) void k_graphs(GraphArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ double red[BLOCK / 64];
  __shared__ int s_slot;
  if (*a.abort) return;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_slot = atomicAdd(a.queue, 1);
    __syncthreads();
    const int slot = s_slot;
    if (slot >= a.num_graphs) break;   // uniform: every thread read the same slot
    solve_graph<BLOCK, RPT>(a, a.order[slot], lds, red, nullptr);
  }
}

// Per-graph statistics of p: sum, #negative, #non-finite; raises *abort if a
// graph's block is not a probability vector.  One workgroup per graph.
__global__ __launch_bounds__(kWG) void k_validate_graphs(const int* __restrict__ graph_ptr,
                                                         const double* __restrict__ p,
                                                         double* __restrict__ rec, int* abort) {
  const int g = blockIdx.x;
  const int v0 = graph_ptr[g], v1 = graph_ptr[g + 1];
  double s = 0.0, neg = 0.0, bad = 0.0;
  for (int u = v0 + threadIdx.x; u < v1; u += kWG) {
    const double v = p[u];
    s += v;
    neg += v < 0.0 ? 1.0 : 0.0;
    bad += isfinite(v) ? 0.0 : 1.0;
  }
  s = block_sum256(s);
  neg = block_sum256(neg);
  bad = block_sum256(bad);
  if (threadIdx.x == 0) {
    double* r = rec + (size_t)g * kRec;
    r[R_PSUM] = s;
    r[R_PNEG] = neg;
    r[R_PBAD] = bad;
    if (bad != 0.0 || neg != 0.0 || !(fabs(s - 1.0) <= 1e-9)) atomicExch(abort, 1);
  }
}

__global__ void k_reset_graph_run(int* abort, int* queue) {
  if (threadIdx.x == 0) *abort = 0;
  if (threadIdx.x < kGraphClasses) queue[threadIdx.x] = 0;
}

}  // namespace

struct GraphRun {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const double* p = nullptr;
  double* x = nullptr;
  double tol = 0.0;
  int block[kGraphClasses] = {};
};

// launch shape: workgroup size and rows per thread
static bool pick_shape(int max_ng, int block, int* rpt) {
  const int need = (max_ng + block - 1) / block;
  static const int opts[] = {1, 2, 3, 4, 5, 6, 8, 10, 16, 20};
  for (int r : opts)
    if (r >= need && !(block == 1024 && r > 10)) {   // as instantiated below
      *rpt = r;
      return true;
    }
  return false;
}

// Instantiated shapes: every workgroup size with every rows-per-thread count
// of pick_shape (1024 threads stop at 10: LDS caps a graph near 10,240 vertices).
#define CPAA_GRAPH_SHAPES(X)                                                              \
  X(64, 1) X(64, 2) X(64, 3) X(64, 4) X(64, 5) X(64, 6) X(64, 8) X(64, 10) X(64, 16)        \
  X(64, 20)                                                                               \
  X(128, 1) X(128, 2) X(128, 3) X(128, 4) X(128, 5) X(128, 6) X(128, 8) X(128, 10)         \
  X(128, 16) X(128, 20)                                                                   \
  X(256, 1) X(256, 2) X(256, 3) X(256, 4) X(256, 5) X(256, 6) X(256, 8) X(256, 10)         \
  X(256, 16) X(256, 20)                                                                   \
  X(512, 1) X(512, 2) X(512, 3) X(512, 4) X(512, 5) X(512, 6) X(512, 8) X(512, 10)         \
  X(512, 16) X(512, 20)                                                                   \
  X(1024, 1) X(1024, 2) X(1024, 3) X(1024, 4) X(1024, 5) X(1024, 6) X(1024, 8)             \
  X(1024, 10)

static hipError_t launch_graphs(int block, int rpt, dim3 grid, size_t lds, hipStream_t st,
                                const GraphArgs& a) {
#define CPAA_G(B, R)                                                              \
  if (block == B && rpt == R) {                                                   \
    hipLaunchKernelGGL((k_graphs<B, R>), grid, dim3(B), lds, st, a);              \
    return hipGetLastError();                                                     \
  }
  CPAA_GRAPH_SHAPES(CPAA_G)
#undef CPAA_G
  return hipErrorInvalidValue;
}

static hipError_t set_lds_limit(int block, int rpt, size_t lds) {
#define CPAA_A(B, R)                                                                       \
  if (block == B && rpt == R)                                                              \
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_graphs<B, R>),              \
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  CPAA_GRAPH_SHAPES(CPAA_A)
#undef CPAA_A
  return hipErrorInvalidValue;
}

// Graph-batch resources hung off the plan's multi-graph workspace.
struct GraphState {
  uint32_t* d_coo = nullptr;
  int* d_coo_off = nullptr;
  int* d_coo_meta = nullptr;
  double* d_rec = nullptr;
  int* d_abort = nullptr;
  double* h_rec = nullptr;
  int num_cus = 0;
  int block[kGraphClasses] = {};   // chosen workgroup size per size class (0 = not chosen yet)
  GraphRun run;
};

static GraphState* state_of(cpaa_plan_s* pl) { return reinterpret_cast<GraphState*>(pl->graph_state); }

void free_graph_state(cpaa_plan_s* pl) {
  GraphState* gs = state_of(pl);
  if (!gs) return;
  if (gs->run.exec) (void)hipGraphExecDestroy(gs->run.exec);
  if (gs->run.graph) (void)hipGraphDestroy(gs->run.graph);
  if (gs->d_coo) (void)hipFree(gs->d_coo);
  if (gs->d_coo_off) (void)hipFree(gs->d_coo_off);
  if (gs->d_coo_meta) (void)hipFree(gs->d_coo_meta);
  if (gs->d_rec) (void)hipFree(gs->d_rec);
  if (gs->d_abort) (void)hipFree(gs->d_abort);
  if (gs->h_rec) (void)hipHostFree(gs->h_rec);
  delete gs;
  pl->graph_state = nullptr;
}

cpaa_status build_graph_state(cpaa_plan_s* pl, const int32_t* rp, const int32_t* ci,
                              const int32_t* gp) {
  GraphState* gs = new (std::nothrow) GraphState();
  if (!gs) {
    set_error("host allocation failed");
    return CPAA_ENOMEM;
  }
  pl->graph_state = gs;
  const int G = pl->num_graphs;
  // per graph: runs of rl entries per lane, rl = nnz_g / 512 rounded up to a
  // multiple of 4 within [4, 16], chunks of 64*rl entries (16-byte aligned),
  // the last one padded
  static_assert(kGraphRunMax % 4 == 0, "runs load four entries at a time");
  std::vector<int> off(G), meta(G);
  size_t total = 0;
  for (int gi = 0; gi < G; ++gi) {
    const int mg = rp[gp[gi + 1]] - rp[gp[gi]];
    const int rl = std::min(kGraphRunMax, std::max(4, ((mg + 511) / 512 + 3) & ~3));
    const int nch = (mg + 64 * rl - 1) / (64 * rl);
    off[gi] = static_cast<int>(total);
    meta[gi] = (nch << 6) | rl;
    total += static_cast<size_t>(nch) * 64 * rl;
  }
  if (total >= (size_t(1) << 31)) {
    set_error("graph batch too large for the packed layout");
    return CPAA_EINVAL;
  }
  std::vector<uint32_t> coo(total, kGraphPad);
  for (int gi = 0; gi < G; ++gi) {
    const int v0 = gp[gi], e0 = rp[v0];
    const int rl = meta[gi] & 63, ch = 64 * rl;
    int q = 0;
    for (int u = gp[gi]; u < gp[gi + 1]; ++u)
      for (int j = rp[u]; j < rp[u + 1]; ++j, ++q) {
        const int c = q / ch, w = q % ch, l = w / rl, i = w % rl;
        coo[off[gi] + static_cast<size_t>(c) * ch + (i >> 2) * 256 + l * 4 + (i & 3)] =
            (static_cast<uint32_t>(u - v0) << 16) | static_cast<uint32_t>(ci[j] - v0);
      }
  }
  if (hipMalloc(&gs->d_coo, std::max<size_t>(coo.size(), 1) * 4) != hipSuccess ||
      hipMalloc(&gs->d_coo_off, (size_t)G * sizeof(int)) != hipSuccess ||
      hipMalloc(&gs->d_coo_meta, (size_t)G * sizeof(int)) != hipSuccess ||
      hipMalloc(&gs->d_rec, (size_t)G * kRec * sizeof(double)) != hipSuccess ||
      hipMalloc(&gs->d_abort, sizeof(int)) != hipSuccess ||
      hipHostMalloc((void**)&gs->h_rec, (size_t)G * kRec * sizeof(double),
                    hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation for the graph batch failed");
    return CPAA_ENOMEM;
  }
  CPAA_HIP(hipMemcpy(gs->d_coo, coo.data(), coo.size() * 4, hipMemcpyHostToDevice));
  CPAA_HIP(hipMemcpy(gs->d_coo_off, off.data(), (size_t)G * sizeof(int), hipMemcpyHostToDevice));
  CPAA_HIP(hipMemcpy(gs->d_coo_meta, meta.data(), (size_t)G * sizeof(int), hipMemcpyHostToDevice));
  hipDeviceProp_t prop;
  CPAA_HIP(hipGetDeviceProperties(&prop, pl->device));
  gs->num_cus = prop.multiProcessorCount;
  return CPAA_OK;
}

// One persistent launch per size class, each with the LDS of its largest
// graph and its own workgroup size (blocks[k]).
struct ClassLaunch {
  GraphArgs a;
  int cls, block, rpt;
  size_t lds;
  dim3 grid;
};

static cpaa_status class_launches(cpaa_plan_s* pl, GraphState* gs, const double* p, double tol,
                                  double* x, const int* blocks, std::vector<ClassLaunch>& out) {
  GraphArgs a;
  a.rp = pl->d_row_ptr;
  a.coo = gs->d_coo;
  a.coo_off = gs->d_coo_off;
  a.coo_meta = gs->d_coo_meta;
  a.graph_ptr = pl->d_graph_ptr;
  a.abort = gs->d_abort;
  a.p = p;
  a.x = x;
  a.c = pl->c;
  a.s = pl->s;
  a.beta = pl->beta;
  a.c0h = pl->ck[0] / 2.0;
  a.tol = tol;
  a.target_main = 0.5 * tol;
  a.target_ref = 0.25 * tol;
  a.k_min = mass_rule_terms(pl, 0.5 * tol);
  a.k_cap_max = pl->opts.k_max > 0 ? std::min(pl->opts.k_max, kMaxTerms) : kMaxTerms;
  a.max_refine = pl->opts.max_refine;
  a.normalize = pl->opts.normalize;
  a.rec = gs->d_rec;
  out.clear();
  for (int k = 0; k < kGraphClasses; ++k) {
    const int count = pl->graph_cls_off[k + 1] - pl->graph_cls_off[k];
    if (count == 0 || blocks[k] == 0) continue;   // 0: left out (tuning runs only)
    ClassLaunch L;
    L.a = a;
    L.a.order = pl->d_graph_order + pl->graph_cls_off[k];
    L.a.num_graphs = count;
    L.a.max_ng = pl->graph_cls_n[k];
    L.a.queue = pl->d_queue + k;
    L.cls = k;
    L.block = blocks[k];
    if (!pick_shape(L.a.max_ng, L.block, &L.rpt)) {
      set_error("graphs too large for the batched kernel");
      return CPAA_EINVAL;
    }
    L.lds = 16 * (size_t)L.a.max_ng;
    // resident workgroups per CU: 2048 threads and 160 KB of LDS per CU
    const int per_cu = std::max(
        1, std::min(2048 / L.block, (int)((160 * 1024) / (L.lds + (size_t)L.block / 8 + 64))));
    L.grid = dim3(std::min(count, gs->num_cus * per_cu));
    out.push_back(L);
  }
  // classes can share a (block, rpt) instantiation: raise its LDS limit to the largest use
  for (const ClassLaunch& L : out) {
    size_t lds = L.lds;
    for (const ClassLaunch& M : out)
      if (M.block == L.block && M.rpt == L.rpt) lds = std::max(lds, M.lds);
    CPAA_HIP(set_lds_limit(L.block, L.rpt, lds));
  }
  return CPAA_OK;
}

// reset the queues -> validate p -> one launch per class, in turn; with
// `ev` (2 kGraphClasses events) class k's launch runs between ev[2k] and ev[2k+1]
static hipError_t enqueue_run(cpaa_plan_s* pl, GraphState* gs, const double* p,
                              const std::vector<ClassLaunch>& launches, hipStream_t st,
                              hipEvent_t* ev = nullptr) {
  hipLaunchKernelGGL(k_reset_graph_run, dim3(1), dim3(64), 0, st, gs->d_abort, pl->d_queue);
  hipLaunchKernelGGL(k_validate_graphs, dim3(pl->num_graphs), dim3(kWG), 0, st,
                     pl->d_graph_ptr, p, gs->d_rec, gs->d_abort);
  hipError_t e = hipGetLastError();
  for (const ClassLaunch& L : launches) {
    if (e == hipSuccess && ev) e = hipEventRecord(ev[2 * L.cls], st);
    if (e == hipSuccess) e = launch_graphs(L.block, L.rpt, L.grid, L.lds, st, L.a);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[2 * L.cls + 1], st);
  }
  return e;
}

static cpaa_status capture_run(cpaa_plan_s* pl, GraphState* gs, const double* p, double tol,
                               double* x, const int* blocks, hipStream_t st) {
  std::vector<ClassLaunch> launches;
  cpaa_status s = class_launches(pl, gs, p, tol, x, blocks, launches);
  if (s != CPAA_OK) return s;
  GraphRun& run = gs->run;
  if (run.exec) (void)hipGraphExecDestroy(run.exec);
  if (run.graph) (void)hipGraphDestroy(run.graph);
  run = GraphRun();
  hipStream_t cs;
  CPAA_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const hipError_t el = enqueue_run(pl, gs, p, launches, cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    if (el != hipSuccess) e = el;
    if (e == hipSuccess) {
      run.graph = graph;
      e = hipGraphInstantiate(&run.exec, graph, nullptr, nullptr, 0);
    } else if (graph) {
      (void)hipGraphDestroy(graph);
    }
  }
  (void)hipStreamDestroy(cs);
  CPAA_HIP(e);
  run.p = p;
  run.x = x;
  run.tol = tol;
  for (int k = 0; k < kGraphClasses; ++k) run.block[k] = blocks[k];
  (void)st;
  return CPAA_OK;
}

// Workgroup size per size class: each candidate runs the whole batch eagerly
// twice (the second timed, class by class); every class keeps its fastest.
// Any workgroup size gives a certified result for every graph.
static cpaa_status tune_blocks(cpaa_plan_s* pl, GraphState* gs, const double* p, double tol,
                               double* x, hipStream_t st) {
  hipEvent_t ev[2 * kGraphClasses] = {};
  hipError_t e = hipSuccess;
  for (int k = 0; k < 2 * kGraphClasses && e == hipSuccess; ++k) e = hipEventCreate(&ev[k]);
  float best[kGraphClasses];
  for (int k = 0; k < kGraphClasses; ++k) {
    best[k] = 1e30f;
    gs->block[k] = 512;
  }
  cpaa_status s = CPAA_OK;
  for (int b : {64, 128, 256, 512, 1024}) {
    if (e != hipSuccess || s != CPAA_OK) break;
    // a class whose largest graph does not fit b threads is left out for b
    int blocks[kGraphClasses];
    bool any = false;
    for (int k = 0; k < kGraphClasses; ++k) {
      int rpt;
      blocks[k] = pick_shape(pl->graph_cls_n[k], b, &rpt) ? b : 0;
      any = any || blocks[k] != 0;
    }
    if (!any) continue;
    std::vector<ClassLaunch> launches;
    if ((s = class_launches(pl, gs, p, tol, x, blocks, launches)) != CPAA_OK) break;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep)
      e = enqueue_run(pl, gs, p, launches, st, rep == 1 ? ev : nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    for (const ClassLaunch& L : launches) {
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[2 * L.cls], ev[2 * L.cls + 1]);
      if (e == hipSuccess && ms < best[L.cls]) {
        best[L.cls] = ms;
        gs->block[L.cls] = b;
      }
    }
  }
  for (int k = 0; k < 2 * kGraphClasses; ++k)
    if (ev[k]) (void)hipEventDestroy(ev[k]);
  CPAA_HIP(e);
  return s;
}

cpaa_status solve_graphs_impl(cpaa_plan_s* pl, const double* p, double tol, double* x,
                              cpaa_report* reps, hipStream_t st) {
  GraphState* gs = state_of(pl);
  if (!gs) {
    set_error("plan has no graph batch");
    return CPAA_EINVAL;
  }
  const int G = pl->num_graphs;
  cpaa_status s;
  // Workgroup size per size class: fixed by the autotuner on the first call,
  // 512 threads otherwise.
  if (gs->block[0] == 0) {
    if (pl->opts.autotune) {
      if ((s = tune_blocks(pl, gs, p, tol, x, st)) != CPAA_OK) return s;
    } else {
      for (int k = 0; k < kGraphClasses; ++k) gs->block[k] = 512;
    }
  }
  GraphRun& run = gs->run;
  bool same = run.exec && run.p == p && run.x == x && run.tol == tol;
  for (int k = 0; k < kGraphClasses; ++k) same = same && run.block[k] == gs->block[k];
  if (!same) {
    if ((s = capture_run(pl, gs, p, tol, x, gs->block, st)) != CPAA_OK) return s;
  }
  CPAA_HIP(hipEventRecord(pl->ev_begin, st));
  CPAA_HIP(hipGraphLaunch(run.exec, st));
  CPAA_HIP(hipEventRecord(pl->ev_end, st));
  CPAA_HIP(hipMemcpyAsync(gs->h_rec, gs->d_rec, (size_t)G * kRec * sizeof(double),
                          hipMemcpyDeviceToHost, st));
  int abort_flag = 0;
  CPAA_HIP(hipMemcpyAsync(&abort_flag, gs->d_abort, sizeof(int), hipMemcpyDeviceToHost, st));
  CPAA_HIP(hipStreamSynchronize(st));
  float ms = 0.f;
  CPAA_HIP(hipEventElapsedTime(&ms, pl->ev_begin, pl->ev_end));
  if (abort_flag) {
    for (int g = 0; g < G; ++g) {
      const double* r = gs->h_rec + (size_t)g * kRec;
      if (r[R_PBAD] != 0.0 || r[R_PNEG] != 0.0 || !(std::fabs(r[R_PSUM] - 1.0) <= 1e-9)) {
        set_error("graph " + std::to_string(g) +
                  ": personalization block must be finite, non-negative and sum to 1");
        return CPAA_EINVAL;
      }
    }
    set_error("personalization rejected");
    return CPAA_EINVAL;
  }
  bool all_ok = true;
  for (int g = 0; g < G; ++g) {
    const double* r = gs->h_rec + (size_t)g * kRec;
    cpaa_report R;
    std::memset(&R, 0, sizeof(R));
    R.terms = static_cast<int32_t>(r[R_TERMS]);
    R.refine_terms = static_cast<int32_t>(r[R_REF_TERMS]);
    R.refinements = static_cast<int32_t>(r[R_REFS]);
    R.cert_bound = r[R_BOUND];
    R.certified = r[R_CERTIFIED] != 0.0;
    R.resid_l1 = r[R_RL1];
    R.resid_max = r[R_RMAX];
    R.mass = r[R_MASS];
    R.series_cert = r[R_SCERT];
    R.ms_total = ms;
    const int64_t gnnz = pl->h_graph_nnz[g];
    R.edges = gnnz * static_cast<int64_t>(R.terms + R.refine_terms);
    all_ok = all_ok && R.certified;
    if (reps) reps[g] = R;
  }
  if (!all_ok) {
    set_error("tolerance not certified for every graph");
    return CPAA_ENOCONV;
  }
  return CPAA_OK;
}

}  // namespace cpaa

using namespace cpaa;

extern "C" cpaa_status cpaa_solve_graphs(cpaa_plan_t pl, const double* p, double tol, double* x,
                                         cpaa_report* reps, void* stream) {
  set_error("");
  if (!pl || !p || !x) {
    set_error("cpaa_solve_graphs: null argument");
    return CPAA_EINVAL;
  }
  if (pl->num_graphs <= 1) {
    set_error("cpaa_solve_graphs needs a block-diagonal plan (num_graphs > 1)");
    return CPAA_EINVAL;
  }
  if (!(tol > 0.0) || !std::isfinite(tol)) {
    set_error("tol must be positive and finite");
    return CPAA_EINVAL;
  }
  if (!pl->opts.io_device) {
    set_error("cpaa_solve_graphs takes device pointers only (io_device = 1)");
    return CPAA_EINVAL;
  }
  return solve_graphs_impl(pl, p, tol, x, reps, reinterpret_cast<hipStream_t>(stream));
}
