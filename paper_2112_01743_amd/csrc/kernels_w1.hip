// Single-vector CPAA kernels (one right-hand side), gfx950.
//
// Hot loop (Alg. 1, Sec. 4.1, in z-space z_k = D^{-1} T_k(P) b; the expansion
// on [a, 1] adds an own-row term and the power method runs on the same kernels
// with other epilogue constants, TermShape):
//     z_{k+1}(u) = 2 * (sum_{v in N(u)} z_k(v)) / d_u - z_{k-1}(u)
//     acc(u)    += c_{k+1} * z_{k+1}(u)                     (FP64)
// (one launch in two or three adds the newest terms at once, from the z_{k-1}
// and z_k it reads anyway: AccUpdate)
// so the SpMV runs on the 0/1 pattern A and the D^{-1} scaling, the
// three-term update, the weighted accumulation and the certificate partial
// d_u |z_{k+1}(u) - beta z_k(u)| all sit in the epilogue of one kernel.
//
// Work decomposition: the plan cuts the CSR into work items of at most
// 256*npt stored entries.  A workgroup loads its item's column indices with
// fully coalesced loads (npt independent loads per thread) and issues npt
// independent gathers per thread, stages the gathered values in LDS, and then
// reduces every row with an adaptive number of lanes per row.  Rows longer
// than one item (hubs of power-law graphs) are cut into chunks over several
// workgroups; chunk sums meet in an FP32 atomic slot and the last arriving
// workgroup runs the row's epilogue.
#include "device.h"
#include "internal.h"

namespace cpaa {
namespace {

// Chunk of a row split over several workgroups: the block's partial sums
// (s, and sa = sum of magnitudes with ABS) go to the row's atomic slot; the
// last arriving block reads the full sums, resets the slot and counter, and
// runs the row's epilogue.
template <typename V, bool ABS, typename Epi>
__device__ __forceinline__ void split_chunk_finish(const WorkItem it, const int* __restrict__ rp,
                                                   V s, V sa, V* __restrict__ split_part,
                                                   int* __restrict__ split_count,
                                                   const int* __restrict__ split_nchunks,
                                                   Epi& epi, V* __restrict__ det_chunk = nullptr,
                                                   int max_chunks = 0, int chunk_cap = 1,
                                                   V* __restrict__ det_defer = nullptr) {
  __shared__ V wsum[4];
  __shared__ V wabs[4];
  const int t = threadIdx.x;
  s = wave_sum(s);
  if (ABS) sa = wave_sum(sa);
  if ((t & 63) == 0) {
    wsum[t >> 6] = s;
    wabs[t >> 6] = sa;
  }
  __syncthreads();
  if (t == 0 && det_chunk != nullptr) {
    // deterministic plans: each chunk publishes its sums in its own slot and the
    // last chunk to arrive adds the chunks in chunk order
    const int slot = -(it.row1 + 1);
    const int c = (it.nnz0 - rp[it.row0]) / chunk_cap;
    V* own = det_chunk + (static_cast<size_t>(slot) * max_chunks + c) * 2;
    __hip_atomic_store(&own[0], (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    if (ABS)
      __hip_atomic_store(&own[1], (wabs[0] + wabs[1]) + (wabs[2] + wabs[3]), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    atomics_done();
    const int nch = split_nchunks[slot];
    const int prev = atomicAdd(&split_count[slot], 1);
    if (prev == nch - 1) {
      atomics_done();
      V full = V(0), full_abs = V(0);
      const V* row_chunks = det_chunk + static_cast<size_t>(slot) * max_chunks * 2;
      for (int q = 0; q < nch; ++q) {
        full += __hip_atomic_load(&row_chunks[2 * q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ABS)
          full_abs += __hip_atomic_load(&row_chunks[2 * q + 1], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
      }
      __hip_atomic_exchange(&split_count[slot], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (det_defer != nullptr) {
        // the row's epilogue (and its share of the block statistics) is left to
        // the grid's last block, which runs the split rows in slot order
        V* d = det_defer + static_cast<size_t>(slot) * 3;
        __hip_atomic_store(&d[0], full, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&d[1], full_abs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&d[2], static_cast<V>(it.row0), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      } else {
        epi.row(it.row0, rp[it.row0 + 1] - rp[it.row0], full, full_abs);
      }
    }
    return;
  }
  if (t == 0) {
    const int slot = -(it.row1 + 1);
    const int ps = ABS ? 2 * slot : slot;
    atomic_add(&split_part[ps], (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]));
    if (ABS) atomic_add(&split_part[ps + 1], (wabs[0] + wabs[1]) + (wabs[2] + wabs[3]));
    atomics_done();
    const int prev = atomicAdd(&split_count[slot], 1);
    if (prev == split_nchunks[slot] - 1) {
      atomics_done();
      const V full = __hip_atomic_exchange(&split_part[ps], V(0), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
      V full_abs = V(0);
      if (ABS)
        full_abs = __hip_atomic_exchange(&split_part[ps + 1], V(0), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_exchange(&split_count[slot], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      epi.row(it.row0, rp[it.row0 + 1] - rp[it.row0], full, full_abs);
    }
  }
}

// Sum of x over N(u) for the rows of one work item; calls
// epi.row(u, d_u, sum, sum_of_magnitudes) exactly once per row, from one thread.
// With ABS the sum of |x| over N(u) is formed too (split partials then use
// two slots per row: [2*slot] sum, [2*slot+1] sum of magnitudes).
template <typename V, int NPT, bool ABS, typename Epi>
__device__ __forceinline__ void spmv_item(const WorkItem it, const int* __restrict__ rp,
                                          const int* __restrict__ ci, const V* __restrict__ x,
                                          V* __restrict__ split_part, int* __restrict__ split_count,
                                          const int* __restrict__ split_nchunks, Epi& epi,
                                          V* __restrict__ det_chunk = nullptr,
                                          int max_chunks = 0, V* __restrict__ det_defer = nullptr) {
  constexpr int CAP = kWG * NPT;
  __shared__ V vals[CAP];
  __shared__ int lrp[kWG * 4 + 1];
  const int t = threadIdx.x;
  const int nb = it.nnz0, ne = it.nnz1;

  int col[NPT];
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    const int j = nb + t + i * kWG;
    col[i] = (j < ne) ? __builtin_nontemporal_load(ci + j) : -1;
  }
  V v[NPT];
#pragma unroll
  for (int i = 0; i < NPT; ++i) v[i] = (col[i] >= 0) ? x[col[i]] : V(0);

  if (it.row1 < 0) {
    // one chunk of a split row
    V s = V(0), sa = V(0);
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      s += v[i];
      if (ABS) sa += fabs(v[i]);
    }
    split_chunk_finish<V, ABS>(it, rp, s, sa, split_part, split_count, split_nchunks, epi,
                               det_chunk, max_chunks, CAP, det_defer);
    return;
  }

#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    const int k = t + i * kWG;
    if (nb + k < ne) vals[k] = v[i];
  }
  const int nrows = it.row1 - it.row0;
  for (int r = t; r <= nrows; r += kWG) lrp[r] = rp[it.row0 + r] - nb;
  __syncthreads();

  const int lpr = nrows >= kWG ? 1 : min(64, prev_pow2(kWG / nrows));
  if (lpr == 1) {
    for (int r = t; r < nrows; r += kWG) {
      const int a = lrp[r], e = lrp[r + 1];
      V s = V(0), sa = V(0);
      int k = a;
      for (; k + 4 <= e; k += 4) {
        s += (vals[k] + vals[k + 1]) + (vals[k + 2] + vals[k + 3]);
        if (ABS) sa += (fabs(vals[k]) + fabs(vals[k + 1])) + (fabs(vals[k + 2]) + fabs(vals[k + 3]));
      }
      for (; k < e; ++k) {
        s += vals[k];
        if (ABS) sa += fabs(vals[k]);
      }
      epi.row(it.row0 + r, e - a, s, sa);
    }
  } else {
    const int sh = __ffs(lpr) - 1;
    const int g = t >> sh, l = t & (lpr - 1);
    V s = V(0), sa = V(0);
    int a = 0, e = 0;
    if (g < nrows) {
      a = lrp[g];
      e = lrp[g + 1];
      for (int k = a + l; k < e; k += lpr) {
        s += vals[k];
        if (ABS) sa += fabs(vals[k]);
      }
    }
    for (int off = lpr >> 1; off > 0; off >>= 1) {
      s += __shfl_xor(s, off);
      if (ABS) sa += __shfl_xor(sa, off);
    }
    if (g < nrows && l == 0) epi.row(it.row0 + g, e - a, s, sa);
  }
}

// Term epilogue in the precision Z of the recurrence (float; double for the
// FP64 debug recurrence); the accumulator and certificate are FP64 always.
template <typename Z>
struct TermEpiT {
  const Z* __restrict__ zc;
  const Z* __restrict__ zp;
  Z* __restrict__ zn;
  double* __restrict__ acc;
  Z alpha, gamma_c, gamma;
  AccUpdate au;
  double beta;
  int want_cert;
  double cert;
  __device__ __forceinline__ bool needs_p() const { return gamma != Z(0) || au.a_prev != 0.0; }
  __device__ __forceinline__ bool needs_c() const {
    return (want_cert && beta != 0.0) || au.a_cur != 0.0 || gamma_c != Z(0);
  }
  __device__ __forceinline__ void row(int r, int d, Z s, Z) {
    const Z p = needs_p() ? zp[r] : Z(0);
    const Z c = needs_c() ? zc[r] : Z(0);
    const double a_old = au.on ? acc[r] : 0.0;
    row_loaded(r, d, s, p, c, a_old);
  }
  // the same with z_{k-1}(r), z_k(r) and acc(r) already loaded (as needed)
  __device__ __forceinline__ void row_loaded(int r, int d, Z s, Z p, Z c, double a_old) {
    Z y = alpha * (s / static_cast<Z>(d));
    if (gamma_c != Z(0)) y -= gamma_c * c;
    if (gamma != Z(0)) y -= gamma * p;
    zn[r] = y;
    if (au.on) {
      // the newest (smallest) term first
      double add = au.a_next * static_cast<double>(y);
      if (au.a_cur != 0.0) add += au.a_cur * static_cast<double>(c);
      if (au.a_prev != 0.0) add += au.a_prev * static_cast<double>(p);
      acc[r] = a_old + add;
    }
    if (want_cert)
      cert += static_cast<double>(d) *
              fabs(static_cast<double>(y) - beta * static_cast<double>(c));
  }
};
using TermEpi = TermEpiT<float>;

template <typename Z>
struct TermArgsT {
  const int* rp;
  const int* ci;
  const WorkItem* items;
  const Z* zc;
  const Z* zp;
  Z* zn;
  double* acc;
  Z alpha, gamma_c, gamma;
  AccUpdate au;
  double beta;
  double* cert;          // [kSlots] or null
  const int* done;       // stop flag or null
  Z* split_part;
  int* split_count;
  const int* split_nchunks;
  int xcd;
};

template <int NPT, typename Z>
__global__ __launch_bounds__(kWG) void k_term_w1(TermArgsT<Z> a) {
  if (a.done != nullptr && *a.done) return;
  const int lb = xcd_logical(blockIdx.x, gridDim.x, a.xcd);
  TermEpiT<Z> epi{a.zc, a.zp, a.zn, a.acc, a.alpha, a.gamma_c, a.gamma, a.au, a.beta,
                  a.cert != nullptr, 0.0};
  spmv_item<Z, NPT, false>(a.items[lb], a.rp, a.ci, a.zc, a.split_part, a.split_count,
                           a.split_nchunks, epi);
  if (a.cert != nullptr) {
    const double s = block_sum256(epi.cert);
    if (threadIdx.x == 0 && s != 0.0) atomic_add(&a.cert[lb % kSlots], s);
  }
}

// ---- column-sliced term ----
// Pass 1 (k_term_sliced): workgroup b runs on XCD b % 8 (the hardware's
// round-robin dispatch) and takes work items of column slice b % 8, so an
// XCD's gathers stay inside one eighth of z_k, which its L2 holds.  Each item
// writes the partial row sums of its rows into part[slice][row] (zeros for
// rows without entries in the slice).  Pass 2 (k_combine_w1) adds the eight
// partials in a fixed order and runs the term epilogue.  The FP64 residual of
// a directed plan runs the same pass over w = D_out^+ x (k_resid_sliced), with
// a second partial per row, the sum of magnitudes its rounding bound needs.
template <typename V>
struct SlicedArgsT {
  const uint32_t* entries;
  const WorkItem* items;
  const int* rp;
  const V* zc;
  V* part;                // [kSlices][n], or [kSlices][n][2] (sum, sum of magnitudes)
  const int* done;
  V* split_part;
  int* split_count;
  const int* split_nchunks;
  int n;
  int item_off[kSlices + 1];
  int slice_off[kSlices + 1];
};
using SlicedArgs = SlicedArgsT<float>;

template <typename V, bool ABS>
struct PartEpi {
  V* __restrict__ out;
  __device__ __forceinline__ void row(int r, int, V s, V sa) {
    if constexpr (ABS) {
      static_assert(sizeof(V) == sizeof(double), "pairs are stored as double2");
      reinterpret_cast<double2*>(out)[r] = make_double2(s, sa);
    } else {
      out[r] = s;
    }
  }
};

template <typename V, bool ABS, int NPT, int RB>
__device__ __forceinline__ void gather_sliced(const SlicedArgsT<V>& a) {
  const int sl = blockIdx.x % kSlices;
  const int k = a.item_off[sl] + static_cast<int>(blockIdx.x / kSlices);
  if (k >= a.item_off[sl + 1]) return;
  const WorkItem it = a.items[k];
  const V* __restrict__ xs = a.zc + a.slice_off[sl];
  PartEpi<V, ABS> epi{a.part + static_cast<size_t>(sl) * a.n * (ABS ? 2 : 1)};
  constexpr uint32_t kNone = kSliceNone;
  const int t = threadIdx.x;
  if (it.row1 < 0) {
    // chunk of a split row: plain local columns
    V sum = V(0), suma = V(0);
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int j = it.nnz0 + t + i * kWG;
      if (j < it.nnz1) {
        const V x = xs[__builtin_nontemporal_load(a.entries + j)];
        sum += x;
        if (ABS) suma += fabs(x);
      }
    }
    split_chunk_finish<V, ABS>(it, a.rp, sum, suma, a.split_part, a.split_count,
                               a.split_nchunks, epi);
    return;
  }
  __shared__ V rsum[kSliceRowsMax];
  __shared__ V rabs[ABS ? kSliceRowsMax : 1];
  __shared__ V hub[ABS ? 1 : kSliceHub];
  const int lane = t & 63;
  const int nrows = it.row1 - it.row0;
  for (int r = t; r < nrows; r += kWG) {
    rsum[r] = V(0);
    if (ABS) rabs[r] = V(0);
  }
  // The slice's first kSliceHub vertices (its highest degrees, the targets of
  // a large share of all gathers) are copied to LDS with coalesced loads.  Not
  // in the FP64 pass with magnitudes: there the LDS copy and its registers
  // would halve the waves per CU (80 KB of LDS, over 256 registers).
  constexpr bool kHub = !ABS;
  const int nhub = kHub ? min(kSliceHub, a.slice_off[sl + 1] - a.slice_off[sl]) : 0;
  for (int c = t; c < nhub; c += kWG) hub[c] = xs[c];
  // Wavefront w owns the logical entries [q0, q0 + Lw); lane l owns the
  // contiguous run [l*RL, (l+1)*RL) of them, stored transposed (element i of
  // the run at physical i*64 + l), so every load below is coalesced while each
  // lane walks its own rows in order.
  const int q0 = (t >> 6) * 64 * NPT;
  const int Lw = min(64 * NPT, (it.nnz1 - it.nnz0) - q0);
  const int RL = Lw > 0 ? (Lw + 63) >> 6 : 0;
  const uint32_t* __restrict__ pe = a.entries + it.nnz0 + q0 + lane;
  uint32_t e[NPT];
#pragma unroll
  for (int i = 0; i < NPT; ++i) e[i] = (i < RL) ? __builtin_nontemporal_load(pe + i * 64) : kNone;
  __syncthreads();
  V v[NPT];
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    V h = V(0), g = V(0);
    const uint32_t c = e[i] >> RB;
    if (kHub && e[i] != kNone && c < static_cast<uint32_t>(kSliceHub)) h = hub[c];
    if (e[i] != kNone && (!kHub || c >= static_cast<uint32_t>(kSliceHub))) g = xs[c];
    v[i] = h + g;
  }
  // Row sums of the run in a register.  A row that starts and ends strictly
  // inside the run has no other contributor: plain store.  The first and the
  // last row of a run may be shared with neighbouring runs: LDS atomic.
  constexpr uint32_t row_mask = (1u << RB) - 1u;
  int row = -1;
  V sum = V(0), suma = V(0);
  bool first = true;
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    if (e[i] != kNone) {
      const int r = static_cast<int>(e[i] & row_mask);
      if (r != row) {
        if (row >= 0) {
          if (first) {
            atomicAdd(&rsum[row], sum);
            if (ABS) atomicAdd(&rabs[row], suma);
          } else {
            rsum[row] = sum;
            if (ABS) rabs[row] = suma;
          }
          first = false;
        }
        row = r;
        sum = v[i];
        if (ABS) suma = fabs(v[i]);
      } else {
        sum += v[i];
        if (ABS) suma += fabs(v[i]);
      }
    }
  }
  // a row that covers every run of the wavefront: one wavefront sum
  const int row_l0 = __builtin_amdgcn_readfirstlane(row);
  if (__all(row == row_l0) && row_l0 >= 0) {
    const V ws = wave_sum(sum);
    V wa = V(0);
    if (ABS) wa = wave_sum(suma);
    if (lane == 0) {
      atomicAdd(&rsum[row_l0], ws);
      if (ABS) atomicAdd(&rabs[row_l0], wa);
    }
  } else if (row >= 0) {
    atomicAdd(&rsum[row], sum);
    if (ABS) atomicAdd(&rabs[row], suma);
  }
  __syncthreads();
  for (int r = t; r < nrows; r += kWG) epi.row(it.row0 + r, 0, rsum[r], ABS ? rabs[r] : V(0));
}

template <int NPT, int RB>
__global__ __launch_bounds__(kWG) void k_term_sliced(SlicedArgs a) {
  if (a.done != nullptr && *a.done) return;
  gather_sliced<float, false, NPT, RB>(a);
}

template <int NPT, int RB>
__global__ __launch_bounds__(kWG) void k_resid_sliced(SlicedArgsT<double> a) {
  gather_sliced<double, true, NPT, RB>(a);
}

struct CombineArgs {
  const int* rp;
  const float* part;
  const float* zc;
  const float* zp;
  float* zn;
  double* acc;
  float alpha, gamma_c, gamma;
  AccUpdate au;
  double beta;
  double* cert;
  const int* done;
  int n;
};

__global__ __launch_bounds__(kWG) void k_combine_w1(CombineArgs a) {
  if (a.done != nullptr && *a.done) return;
  TermEpi epi{a.zc, a.zp, a.zn, a.acc, a.alpha, a.gamma_c, a.gamma, a.au, a.beta,
              a.cert != nullptr, 0.0};
  const size_t n = static_cast<size_t>(a.n);
  for (int u = blockIdx.x * kWG + threadIdx.x; u < a.n; u += gridDim.x * kWG) {
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kSlices; ++k) s += a.part[k * n + u];
    epi.row(u, a.rp[u + 1] - a.rp[u], s, 0.f);
  }
  if (a.cert != nullptr) {
    const double c = block_sum256(epi.cert);
    if (threadIdx.x == 0 && c != 0.0) atomic_add(&a.cert[blockIdx.x % kSlots], c);
  }
}

// ---- hub-sliced term (undirected plans; layout in internal.h) ----
// Pass 1 (k_term_hub): workgroup b serves column slice b % 8 (the XCD the
// hardware places it on, so the slice's part of z_k stays in that XCD's L2),
// copies the slice's first HUB vertices to LDS once for its WAVES wavefronts,
// and each wavefront sums one wave item.  Gathers of hub columns read LDS, the
// rest read the slice in L2.  Row sums are formed without atomics and in a
// fixed order: each lane sums the rows of its run in a register, rows inside
// the run are complete, and the rows that cross lane boundaries are finished
// by a segmented scan over the lanes (Hillis-Steele, keyed by row), so every
// present row is written once, in LDS, and then copied out coalesced.
// Pass 2 (k_combine_hub) adds a row's partials in slice order and runs the
// term epilogue.  With V = double the same pass sums acc for the FP64
// residual (pass 2 is then k_resid_hub).
template <typename V>
struct HubArgsT {
  const uint32_t* entries;
  const HubItem* items;
  const V* zc;             // the vector gathered (z_k; acc for the FP64 residual)
  V* part;                 // [pofs[kSlices]]
  const int* done;
  V* chunk_val;
  int* long_cnt;
  const int* chunk_long;
  const int* long_first;
  const int* long_nch;
  const int* long_out;
  int item_off[kSlices + 1];
  int slice_off[kSlices + 1];
  int pofs[kSlices + 1];
};
using HubArgs = HubArgsT<float>;

// ordering of LDS accesses between the lanes of one wavefront
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int WAVES, int HUB, typename V = float>
__global__ __launch_bounds__(WAVES * 64) void k_term_hub(HubArgsT<V> a) {
  if (a.done != nullptr && *a.done) return;
  static_assert((WAVES * kHubRowsPad + HUB) * sizeof(V) <= 160 * 1024, "LDS of one workgroup");
  __shared__ V hub[HUB];
  __shared__ V rsum[WAVES][kHubRowsPad];
  const int sl = blockIdx.x % kSlices;
  const int grp = blockIdx.x / kSlices;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nk = a.item_off[sl + 1] - a.item_off[sl];
  if (grp * WAVES >= nk) return;   // past the slice's last item (whole workgroup)
  const int lo = a.slice_off[sl];
  const V* __restrict__ xs = a.zc + lo;
  const int nh = min(HUB, a.slice_off[sl + 1] - lo);
  if constexpr (sizeof(V) == 4) {
    // 16-byte loads for the 16-byte-aligned body of the hub, scalar head and tail
    const int head = min(nh, (4 - (lo & 3)) & 3);
    const int body = (nh - head) & ~3;
    if (static_cast<int>(threadIdx.x) < head) hub[threadIdx.x] = xs[threadIdx.x];
    const float4* __restrict__ src4 = reinterpret_cast<const float4*>(xs + head);
    for (int c = threadIdx.x; c < body / 4; c += WAVES * 64) {
      const float4 v = src4[c];
      hub[head + 4 * c] = v.x;
      hub[head + 4 * c + 1] = v.y;
      hub[head + 4 * c + 2] = v.z;
      hub[head + 4 * c + 3] = v.w;
    }
    for (int c = head + body + threadIdx.x; c < nh; c += WAVES * 64) hub[c] = xs[c];
  } else {
    for (int c = threadIdx.x; c < nh; c += WAVES * 64) hub[c] = xs[c];
  }
  __syncthreads();
  const HubItem* __restrict__ items = a.items + a.item_off[sl];
  V* __restrict__ part = a.part + a.pofs[sl];
  V* rs = rsum[wv];
  constexpr uint32_t kNone = kSliceNone;
  constexpr uint32_t row_mask = (1u << kHubRowBits) - 1u;
  const int k = grp * WAVES + wv;
  if (k < nk) {
    const HubItem it = items[k];
    if (it.rows < 0) {
      // chunk of a long row: plain local columns, one wavefront sum
      V sum = 0;
#pragma unroll
      for (int i = 0; i < kHubNpt; ++i) {
        const int j = lane + i * 64;
        if (j < it.len) {
          const uint32_t c = __builtin_nontemporal_load(a.entries + it.e0 + j);
          sum += c < static_cast<uint32_t>(HUB) ? hub[c] : xs[c];
        }
      }
      sum = wave_sum(sum);
      if (lane == 0) {
        // publish the chunk sum, then count the arrival; the last chunk adds
        // all chunk sums in chunk order (fixed order whatever the arrivals)
        const int slot = -(it.rows + 1);
        __hip_atomic_exchange(&a.chunk_val[slot], sum, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
        atomics_done();
        const int lr = a.chunk_long[slot];
        const int prev = atomicAdd(&a.long_cnt[lr], 1);
        if (prev == a.long_nch[lr] - 1) {
          atomics_done();
          const int f = a.long_first[lr], nc = a.long_nch[lr];
          V tot = 0;
          for (int q = 0; q < nc; ++q)
            tot += __hip_atomic_exchange(&a.chunk_val[f + q], V(0), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_exchange(&a.long_cnt[lr], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          a.part[a.long_out[lr]] = tot;
        }
      }
      return;
    }
    const int RL = hub_run_length(it.len);
    const int rl = max(0, min(RL, it.len - lane * RL));   // entries of this lane's run
    // four consecutive run elements per 16-byte load (hub_slot layout)
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4* __restrict__ pe4 = reinterpret_cast<const u32x4*>(a.entries + it.e0) + lane;
    uint32_t e[kHubNpt];
#pragma unroll
    for (int q = 0; q < kHubNpt / 4; ++q) {
      const u32x4 v = (4 * q < RL) ? __builtin_nontemporal_load(pe4 + q * 64)
                                   : u32x4{kNone, kNone, kNone, kNone};
      e[4 * q] = v.x;
      e[4 * q + 1] = v.y;
      e[4 * q + 2] = v.z;
      e[4 * q + 3] = v.w;
    }
    // Present rows of an item are consecutive and each has an entry, so along
    // a run the row rises by exactly one where a new row starts: the run's
    // first row and a bit mask of row starts replace the packed entries once
    // the gathers are issued.
    const int fr = rl > 0 ? static_cast<int>(e[0] & row_mask) : -1;
    uint32_t starts = 0;
#pragma unroll
    for (int i = 1; i < kHubNpt; ++i)
      if (i < rl && ((e[i] ^ e[i - 1]) & row_mask) != 0) starts |= 1u << i;
    V v[kHubNpt];
#pragma unroll
    for (int i = 0; i < kHubNpt; ++i) {
      const uint32_t c = e[i] >> kHubRowBits;
      V h = 0, g = 0;
      if (i < rl && c < static_cast<uint32_t>(HUB)) h = hub[c];
      if (i < rl && c >= static_cast<uint32_t>(HUB)) g = xs[c];
      v[i] = h + g;
    }
    // rows of the run: the first (fr, fs) and last (lr, ls) may continue in the
    // neighbouring lanes; rows strictly between are complete here.  Every
    // finished row is stored; the first row's store is overwritten below with
    // its complete sum by this same lane.  (v[i] = 0 past the run.)
    int row = fr;
    V fs = 0, cur = v[0];
#pragma unroll
    for (int i = 1; i < kHubNpt; ++i) {
      const bool st = (starts >> i) & 1u;
      if (st) rs[row + (row >> 5)] = cur;
      fs = (st && row == fr) ? cur : fs;
      row += st ? 1 : 0;
      cur = st ? v[i] : cur + v[i];
    }
    const int lr = row;
    const V ls = cur;
    if (fr == lr) fs = ls;
    // segmented inclusive scan of the last-row sums over the lanes (rows
    // ascend with the lane, so equal keys are contiguous); empty lanes get
    // keys of their own
    const int key = rl > 0 ? lr : -2 - lane;
    V S = rl > 0 ? ls : V(0);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const V So = __shfl_up(S, off);
      const int ko = __shfl_up(key, off);
      if (lane >= off && ko == key) S = So + S;
    }
    const int key_prev = __shfl_up(key, 1);
    const V S_prev = __shfl_up(S, 1);
    const int fr_next = __shfl_down(rl > 0 ? fr : -1, 1);
    if (rl > 0) {
      if (fr != lr) rs[fr + (fr >> 5)] = (lane > 0 && key_prev == fr) ? S_prev + fs : fs;
      if (lane == 63 || fr_next != lr) rs[lr + (lr >> 5)] = S;
    }
    wave_lds_sync();
    for (int r = lane; r < it.rows; r += 64) part[it.j0 + r] = rs[r + (r >> 5)];
  }
}

struct HubCombineArgs {
  double* det_part;       // deterministic plans: per-block certificate partials, else null
  int* det_count;
  const int* rp;
  const uint8_t* mask;
  const int* base;        // [ceil(n/64)][kSlices]
  const float* part;
  int pofs[kSlices];
  const float* zc;
  const float* zp;
  float* zn;
  double* acc;
  float alpha, gamma_c, gamma;
  AccUpdate au;
  double beta;
  double* cert;
  const int* done;
  int n;
};

__global__ __launch_bounds__(kWG) void k_combine_hub(HubCombineArgs a) {
  if (a.done != nullptr && *a.done) return;
  TermEpi epi{a.zc, a.zp, a.zn, a.acc, a.alpha, a.gamma_c, a.gamma, a.au, a.beta,
              a.cert != nullptr, 0.0};
  // one row per thread, one 64-row block per wavefront (grid covers n)
  const int lane = threadIdx.x & 63;
  const uint64_t below = (uint64_t(1) << lane) - 1;
  const int blk = __builtin_amdgcn_readfirstlane(static_cast<int>(
      blockIdx.x * (kWG / 64) + (threadIdx.x >> 6)));
  const int u = blk * 64 + lane;
  if (blk * 64 < a.n) {
    // the row's own inputs are loaded first, so they are in flight together
    // with the partials (whose addresses need the mask and the block bases)
    const bool in = u < a.n;
    const int d = in ? a.rp[u + 1] - a.rp[u] : 1;
    const float p = in && epi.needs_p() ? a.zp[u] : 0.f;
    const float c = in && epi.needs_c() ? a.zc[u] : 0.f;
    const double a_old = in && a.au.on ? a.acc[u] : 0.0;
    const uint32_t m = in ? a.mask[u] : 0u;
    const int* __restrict__ bs = a.base + static_cast<size_t>(blk) * kSlices;
    int idx[kSlices];
#pragma unroll
    for (int sl = 0; sl < kSlices; ++sl) {
      const bool bit = (m >> sl) & 1u;
      idx[sl] = bit ? a.pofs[sl] + bs[sl] + __popcll(__ballot(bit) & below) : -1;
    }
    float pv[kSlices];
#pragma unroll
    for (int sl = 0; sl < kSlices; ++sl) pv[sl] = idx[sl] >= 0 ? a.part[idx[sl]] : 0.f;
    float s = 0.f;
#pragma unroll
    for (int sl = 0; sl < kSlices; ++sl)
      if (idx[sl] >= 0) s += pv[sl];
    if (in) epi.row_loaded(u, d, s, p, c, a_old);
  }
  if (a.cert != nullptr) {
    double c[1] = {block_sum256(epi.cert)};
    if (a.det_part != nullptr) {
      if (ordered_block_sum<1>(c, blockIdx.x, gridDim.x, a.det_part, a.det_count) &&
          threadIdx.x == 0)
        atomic_add(&a.cert[0], c[0]);
    } else if (threadIdx.x == 0 && c[0] != 0.0) {
      atomic_add(&a.cert[blockIdx.x % kSlots], c[0]);
    }
  }
}

struct ResidEpi {
  const double* __restrict__ acc;
  const double* __restrict__ b;
  double* __restrict__ r_out;
  double c;
  double f_abs, f_max, f_q, f_mass, f_round, f_bad;
  // r = b - d a + c s.  Besides |r| the row adds an upper bound on the FP64
  // rounding error of that evaluation (any summation order):
  // (d + 3) u (|b| + d |a| + c sum|a_v|), u = 2^-53, which keeps
  // ||r||_1 / (1-c) a rigorous bound for the x actually returned.
  __device__ __forceinline__ void row(int r, int d, double s, double sa) {
    const double a = acc[r];
    const double dd = static_cast<double>(d);
    const double bb = b[r];
    const double res = bb - dd * a + c * s;
    r_out[r] = res;
    const double ar = fabs(res);
    if (!isfinite(res)) f_bad += 1.0;
    f_abs += ar;
    f_max = fmax(f_max, ar);
    f_q += res * res / dd;
    f_mass += dd * a;
    f_round += (dd + 3.0) * 0x1p-53 * (fabs(bb) + dd * fabs(a) + c * sa);
  }
};

struct ResidArgs {
  const int* rp;
  const int* ci;
  const WorkItem* items;
  const double* acc;
  const double* b;
  double* r;
  double c;
  double* stat_slots;   // [kSlots][1][kStat]
  double* split_part;
  int* split_count;
  const int* split_nchunks;
  int xcd;
  double* det_part;     // deterministic plans: per-block statistics, else null
  int* det_count;
  double* det_chunk;    // deterministic plans: per-chunk sums of split rows
  int max_chunks;
  double* det_defer;    // deterministic plans: [split rows][3] full sums and row, left to the
                        // last block
  int n_split;
};

template <int NPT>
__global__ __launch_bounds__(kWG) void k_resid_w1(ResidArgs a) {
  const int lb = xcd_logical(blockIdx.x, gridDim.x, a.xcd);
  ResidEpi epi{a.acc, a.b, a.r, a.c, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const bool det = a.det_part != nullptr;
  spmv_item<double, NPT, true>(a.items[lb], a.rp, a.ci, a.acc, a.split_part, a.split_count,
                               a.split_nchunks, epi, det ? a.det_chunk : nullptr, a.max_chunks,
                               det ? a.det_defer : nullptr);
  double sums[4] = {block_sum256(epi.f_abs), block_sum256(epi.f_q), block_sum256(epi.f_mass),
                    block_sum256(epi.f_round)};
  const double s_max = block_max256(epi.f_max);
  const double s_bad = block_sum256(epi.f_bad);
  if (det) {
    // deterministic plans: real-valued sums in block order; the maximum and the
    // count of non-finite rows are exact in any order.  The last block also runs
    // the epilogue of the split rows, in slot order, and adds their statistics
    // after the blocks'.
    if (threadIdx.x == 0) {
      atomic_max_nonneg(&a.stat_slots[1], s_max);
      if (s_bad != 0.0) atomic_add(&a.stat_slots[5], s_bad);
    }
    if (!ordered_block_sum<4>(sums, lb, gridDim.x, a.det_part, a.det_count)) return;
    ResidEpi e{a.acc, a.b, a.r, a.c, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int slot = threadIdx.x; slot < a.n_split; slot += kWG) {
      const double* d = a.det_defer + static_cast<size_t>(slot) * 3;
      const double sv = __hip_atomic_load(&d[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const double sa = __hip_atomic_load(&d[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int row = static_cast<int>(
          __hip_atomic_load(&d[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      e.row(row, a.rp[row + 1] - a.rp[row], sv, sa);
    }
    const double x_abs = block_sum256(e.f_abs), x_q = block_sum256(e.f_q);
    const double x_mass = block_sum256(e.f_mass), x_round = block_sum256(e.f_round);
    const double x_max = block_max256(e.f_max), x_bad = block_sum256(e.f_bad);
    if (threadIdx.x == 0) {
      atomic_add(&a.stat_slots[0], sums[0] + x_abs);
      atomic_add(&a.stat_slots[2], sums[1] + x_q);
      atomic_add(&a.stat_slots[3], sums[2] + x_mass);
      atomic_add(&a.stat_slots[4], sums[3] + x_round);
      atomic_max_nonneg(&a.stat_slots[1], x_max);
      if (x_bad != 0.0) atomic_add(&a.stat_slots[5], x_bad);
    }
    return;
  }
  const double s_abs = sums[0], s_q = sums[1], s_mass = sums[2], s_round = sums[3];
  if (threadIdx.x == 0) {
    double* o = a.stat_slots + (size_t)(lb % kSlots) * kStat;
    atomic_add(&o[0], s_abs);
    atomic_max_nonneg(&o[1], s_max);
    atomic_add(&o[2], s_q);
    atomic_add(&o[3], s_mass);
    atomic_add(&o[4], s_round);
    if (s_bad != 0.0) atomic_add(&o[5], s_bad);
  }
}

// FP64 residual of hub-sliced plans, pass 2 (pass 1 is k_term_hub<..., double>
// on acc, leaving each row's partial sums of acc over its neighbours per
// slice): r = b - d a + c s per row with s the partials added in slice order,
// and the statistics of k_resid_w1; optionally also x = D acc, the result as
// it stands (what the finalize kernel would write with scale 1).  The rounding bound is the same sum,
// regrouped: sum_u (d_u + 3) u (|b_u| + d_u |a_u| + c sum_{v in N(u)} |a_v|)
// = sum_u (d_u + 3) u (|b_u| + d_u |a_u|) + c u sum_v |a_v| w_v, with the
// plan's w_v = sum_{u in N(v)} (d_u + 3), so no sum of |a_v| is gathered.
struct ResidHubArgs {
  const int* rp;
  const uint8_t* mask;
  const int* base;        // [ceil(n/64)][kSlices]
  const double* part;
  int pofs[kSlices];
  const double* acc;
  const double* b;
  const double* wround;
  double* r;
  const int* perm;        // caller's label of each row
  double* x;              // x = D acc written at the caller's labels, or null
  double c;
  double* stat_slots;     // [kSlots][1][kStat]
  double* det_part;       // deterministic plans: per-block statistics, else null
  int* det_count;
  int n;
};

__global__ __launch_bounds__(kWG) void k_resid_hub(ResidHubArgs a) {
  constexpr double u53 = 0x1p-53;
  double f_abs = 0.0, f_max = 0.0, f_q = 0.0, f_mass = 0.0, f_round = 0.0, f_bad = 0.0;
  const int lane = threadIdx.x & 63;
  const uint64_t below = (uint64_t(1) << lane) - 1;
  const int blk = __builtin_amdgcn_readfirstlane(static_cast<int>(
      blockIdx.x * (kWG / 64) + (threadIdx.x >> 6)));
  const int u = blk * 64 + lane;
  if (blk * 64 < a.n) {
    const bool in = u < a.n;
    const int d = in ? a.rp[u + 1] - a.rp[u] : 1;
    const double acc = in ? a.acc[u] : 0.0;
    const double bb = in ? a.b[u] : 0.0;
    const double w = in ? a.wround[u] : 0.0;
    const uint32_t m = in ? a.mask[u] : 0u;
    const int* __restrict__ bs = a.base + static_cast<size_t>(blk) * kSlices;
    int idx[kSlices];
#pragma unroll
    for (int sl = 0; sl < kSlices; ++sl) {
      const bool bit = (m >> sl) & 1u;
      idx[sl] = bit ? a.pofs[sl] + bs[sl] + __popcll(__ballot(bit) & below) : -1;
    }
    double pv[kSlices];
#pragma unroll
    for (int sl = 0; sl < kSlices; ++sl) pv[sl] = idx[sl] >= 0 ? a.part[idx[sl]] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int sl = 0; sl < kSlices; ++sl)
      if (idx[sl] >= 0) s += pv[sl];
    if (in) {
      const double dd = static_cast<double>(d);
      const double res = bb - dd * acc + a.c * s;
      a.r[u] = res;
      if (a.x != nullptr) a.x[a.perm[u]] = dd * acc;
      const double ar = fabs(res);
      if (!isfinite(res)) f_bad += 1.0;
      f_abs += ar;
      f_max = fmax(f_max, ar);
      f_q += res * res / dd;
      f_mass += dd * acc;
      f_round += (dd + 3.0) * u53 * (fabs(bb) + dd * fabs(acc)) + a.c * u53 * fabs(acc) * w;
    }
  }
  double sums[4] = {block_sum256(f_abs), block_sum256(f_q), block_sum256(f_mass),
                    block_sum256(f_round)};
  const double s_max = block_max256(f_max);
  const double s_bad = block_sum256(f_bad);
  if (a.det_part != nullptr) {
    // deterministic plans: real-valued sums in block order; the maximum and the
    // count of non-finite rows are exact in any order
    if (threadIdx.x == 0) {
      atomic_max_nonneg(&a.stat_slots[1], s_max);
      if (s_bad != 0.0) atomic_add(&a.stat_slots[5], s_bad);
    }
    if (ordered_block_sum<4>(sums, blockIdx.x, gridDim.x, a.det_part, a.det_count) &&
        threadIdx.x == 0) {
      atomic_add(&a.stat_slots[0], sums[0]);
      atomic_add(&a.stat_slots[2], sums[1]);
      atomic_add(&a.stat_slots[3], sums[2]);
      atomic_add(&a.stat_slots[4], sums[3]);
    }
    return;
  }
  if (threadIdx.x == 0) {
    double* o = a.stat_slots + (size_t)(blockIdx.x % kSlots) * kStat;
    atomic_add(&o[0], sums[0]);
    atomic_max_nonneg(&o[1], s_max);
    atomic_add(&o[2], sums[1]);
    atomic_add(&o[3], sums[2]);
    atomic_add(&o[4], sums[3]);
    if (s_bad != 0.0) atomic_add(&o[5], s_bad);
  }
}

// z_0 = b / d (FP32), acc (+)= (c_0/2) b / d (FP64), b = scale * src.
// Statistics: [0] sum src, [2] sum b^2/d, [4] #negative src, [5] #non-finite src.
template <typename Z>
__global__ __launch_bounds__(kWG) void k_init_w1(int n, const int* __restrict__ rp,
                                                 const int* __restrict__ perm,
                                                 const double* __restrict__ src, double scale,
                                                 int add, int store_b, int series, double c0h,
                                                 double* __restrict__ b, Z* __restrict__ z0,
                                                 double* __restrict__ acc,
                                                 double* __restrict__ stat_slots,
                                                 double* __restrict__ det_part,
                                                 int* __restrict__ det_count) {
  double f_sum = 0, f_q = 0, f_neg = 0, f_bad = 0;
  for (int u = blockIdx.x * kWG + threadIdx.x; u < n; u += gridDim.x * kWG) {
    const double p = src[perm ? perm[u] : u];
    const double bu = scale * p;
    const double d = static_cast<double>(rp[u + 1] - rp[u]);
    const double y = bu / d;
    if (store_b) b[u] = bu;
    if (series) {
      z0[u] = static_cast<Z>(y);
      acc[u] = add ? acc[u] + c0h * y : c0h * y;
    }
    f_sum += p;
    f_q += bu * y;
    f_neg += (p < 0.0) ? 1.0 : 0.0;
    f_bad += isfinite(p) ? 0.0 : 1.0;
  }
  double sums[2] = {block_sum256(f_sum), block_sum256(f_q)};
  const double s4 = block_sum256(f_neg), s5 = block_sum256(f_bad);
  if (det_part != nullptr) {
    // deterministic plans: the real-valued sums in block order (the counts are
    // exact in any order)
    if (ordered_block_sum<2>(sums, blockIdx.x, gridDim.x, det_part, det_count) &&
        threadIdx.x == 0) {
      atomic_add(&stat_slots[0], sums[0]);
      atomic_add(&stat_slots[2], sums[1]);
    }
    if (threadIdx.x == 0) {
      if (s4 != 0.0) atomic_add(&stat_slots[4], s4);
      if (s5 != 0.0) atomic_add(&stat_slots[5], s5);
    }
    return;
  }
  if (threadIdx.x == 0) {
    double* o = stat_slots + (size_t)(blockIdx.x % kSlots) * kStat;
    atomic_add(&o[0], sums[0]);
    atomic_add(&o[2], sums[1]);
    if (s4 != 0.0) atomic_add(&o[4], s4);
    if (s5 != 0.0) atomic_add(&o[5], s5);
  }
}

// acc = x0 / d; statistic [1] counts non-finite x0 entries.
__global__ __launch_bounds__(kWG) void k_load_x0_w1(int n, const int* __restrict__ rp,
                                                    const int* __restrict__ perm,
                                                    const double* __restrict__ x0,
                                                    double* __restrict__ acc,
                                                    double* __restrict__ stat_slots) {
  double f_bad = 0;
  for (int u = blockIdx.x * kWG + threadIdx.x; u < n; u += gridDim.x * kWG) {
    const double v = x0[perm ? perm[u] : u];
    f_bad += isfinite(v) ? 0.0 : 1.0;
    acc[u] = v / static_cast<double>(rp[u + 1] - rp[u]);
  }
  const double s5 = block_sum256(f_bad);
  if (threadIdx.x == 0 && s5 != 0.0)
    atomic_add(&stat_slots[(size_t)(blockIdx.x % kSlots) * kStat + 1], s5);
}

// x = scale * D acc
__global__ __launch_bounds__(kWG) void k_finalize_w1(int n, const int* __restrict__ rp,
                                                     const int* __restrict__ perm,
                                                     const double* __restrict__ acc, double scale,
                                                     double* __restrict__ x) {
  for (int u = blockIdx.x * kWG + threadIdx.x; u < n; u += gridDim.x * kWG)
    x[perm ? perm[u] : u] = scale * static_cast<double>(rp[u + 1] - rp[u]) * acc[u];
}

int elem_grid(int64_t n) {
  const int64_t g = (n + kWG - 1) / kWG;
  return static_cast<int>(g < 8192 ? (g < 1 ? 1 : g) : 8192);
}

// ---------------------------------------------------------------------------
// Directed graphs (Sec. 2.1): row u lists the v with v -> u, P = A D_out^+ on
// the columns with out-edges and P' = P + p d^T sends a dangling vertex's mass
// along p.  The power method x_{t+1} = cP'x_t + (1-c)p runs in x-space as x_0
// plus its increments delta_t = (cP')^t delta_0, delta_0 = c(P' - I)x_0:
//     delta_{t+1}(u) = c sum_{v -> u} delta_t(v)/dout_v + c m_t p_u,
// m_t the dangling mass of delta_t.  The SpMV gathers z_t = D_out^+ delta_t
// (FP32, zero at dangling vertices); m_t is reduced into dang[buffer of z_t]
// by the launch that forms delta_t and read by the next one.
// ---------------------------------------------------------------------------

// Sum of kSlots (= 64) reduction slots by the first wavefront, one per lane;
// the result is valid in every lane of that wavefront.
static_assert(kSlots == 64, "one slot per lane");
__device__ __forceinline__ double slot_sum(const double* __restrict__ slots) {
  return wave_sum(slots[threadIdx.x & 63]);
}

// acc (+)= x_0 = scale * src; z_0 = D_out^+ x_0; dangling mass of x_0 -> dang0.
__global__ __launch_bounds__(kWG) void k_init_dir(int n, const int* __restrict__ dout,
                                                  const int* __restrict__ perm,
                                                  const double* __restrict__ src, double scale,
                                                  double one_minus_c, int add, int store_b,
                                                  double* __restrict__ b, float* __restrict__ z0,
                                                  double* __restrict__ acc,
                                                  double* __restrict__ dang0,
                                                  double* __restrict__ stat_slots) {
  double f_sum = 0, f_neg = 0, f_bad = 0, f_dang = 0;
  for (int u = blockIdx.x * kWG + threadIdx.x; u < n; u += gridDim.x * kWG) {
    const double p = src[perm ? perm[u] : u];
    const double x = scale * p;
    const int d = dout[u];
    if (store_b) b[u] = one_minus_c * p;
    z0[u] = d > 0 ? static_cast<float>(x / d) : 0.f;
    acc[u] = add ? acc[u] + x : x;
    if (d == 0) f_dang += x;
    f_sum += p;
    f_neg += (p < 0.0) ? 1.0 : 0.0;
    f_bad += isfinite(p) ? 0.0 : 1.0;
  }
  const double s0 = block_sum256(f_sum), s4 = block_sum256(f_neg);
  const double s5 = block_sum256(f_bad), sd = block_sum256(f_dang);
  if (threadIdx.x == 0) {
    double* o = stat_slots + (size_t)(blockIdx.x % kSlots) * kStat;
    atomic_add(&o[0], s0);
    if (s4 != 0.0) atomic_add(&o[4], s4);
    if (s5 != 0.0) atomic_add(&o[5], s5);
    if (sd != 0.0) atomic_add(&dang0[blockIdx.x % kSlots], sd);
  }
}

struct DirTermEpi {
  const double* __restrict__ b;      // (1-c) p
  const double* __restrict__ x0;     // first launch only: x_0 = x0_scale * x0
  const int* __restrict__ dout;
  float* __restrict__ zn;
  double* __restrict__ acc;
  double c, m, p_scale, x0_scale;
  int want_cert;
  double cert, mnext;
  __device__ __forceinline__ void row(int r, int, float s, float) {
    double y = c * static_cast<double>(s) + c * m * (p_scale * b[r]);
    if (x0 != nullptr) y -= c * x0_scale * x0[r];
    const int d = dout[r];
    zn[r] = d > 0 ? static_cast<float>(y / d) : 0.f;
    acc[r] += y;
    if (d == 0) mnext += y;
    // (1-c)|delta|, the scale of the undirected power method's certificate
    if (want_cert) cert += (1.0 - c) * fabs(y);
  }
};

struct DirArgs {
  const int* rp;
  const int* ci;
  const WorkItem* items;
  const int* dout;
  const double* b;
  const double* x0;
  double x0_scale;
  const float* zc;
  float* zn;
  double* acc;
  const double* dang_cur;   // [kSlots] dangling mass of the increment in zc
  double* dang_next;        // [kSlots] of the increment this launch forms (zero on entry)
  double* dang_clear;       // [kSlots] cleared here for the launch after next
  double c;
  double* cert;
  const int* done;
  float* split_part;
  int* split_count;
  const int* split_nchunks;
  int xcd;
};

template <int NPT>
__global__ __launch_bounds__(kWG) void k_term_dir(DirArgs a) {
  if (a.done != nullptr && *a.done) return;
  __shared__ double m_sh;
  if (threadIdx.x < 64) {
    const double m = slot_sum(a.dang_cur);
    if (threadIdx.x == 0) m_sh = m;
  }
  if (blockIdx.x == 0 && threadIdx.x < kSlots) a.dang_clear[threadIdx.x] = 0.0;
  __syncthreads();
  const int lb = xcd_logical(blockIdx.x, gridDim.x, a.xcd);
  DirTermEpi epi{a.b, a.x0, a.dout, a.zn, a.acc, a.c, m_sh, 1.0 / (1.0 - a.c), a.x0_scale,
                 a.cert != nullptr, 0.0, 0.0};
  spmv_item<float, NPT, false>(a.items[lb], a.rp, a.ci, a.zc, a.split_part, a.split_count,
                               a.split_nchunks, epi);
  const double cs = block_sum256(epi.cert);
  const double ms = block_sum256(epi.mnext);
  if (threadIdx.x == 0) {
    if (a.cert != nullptr && cs != 0.0) atomic_add(&a.cert[lb % kSlots], cs);
    if (ms != 0.0) atomic_add(&a.dang_next[lb % kSlots], ms);
  }
}

// w = D_out^+ x for the residual; dangling mass of x and of |x| -> dx, dxa.
__global__ __launch_bounds__(kWG) void k_dir_w(int n, const int* __restrict__ dout,
                                               const double* __restrict__ acc,
                                               double* __restrict__ w, double* __restrict__ dx,
                                               double* __restrict__ dxa) {
  double f = 0, fa = 0;
  for (int u = blockIdx.x * kWG + threadIdx.x; u < n; u += gridDim.x * kWG) {
    const int d = dout[u];
    const double x = acc[u];
    w[u] = d > 0 ? x / d : 0.0;
    if (d == 0) {
      f += x;
      fa += fabs(x);
    }
  }
  const double s = block_sum256(f), sa = block_sum256(fa);
  if (threadIdx.x == 0) {
    if (s != 0.0) atomic_add(&dx[blockIdx.x % kSlots], s);
    if (sa != 0.0) atomic_add(&dxa[blockIdx.x % kSlots], sa);
  }
}

// r = b - x + c (A w) + c m_x p, with an upper bound on the FP64 rounding of
// its evaluation: (k + 5) u (|b| + |x| + c sum|w_v| + c |m_x| p) for a row of
// k entries (w_v = x_v/dout_v adds one rounding each), plus the rounding of the
// n-term sum m_x: c p n u sum|x_dangling|.
struct DirResidEpi {
  const double* __restrict__ acc;
  const double* __restrict__ b;
  double* __restrict__ r_out;
  double c, mx, mxa, p_scale, nu;
  double f_abs, f_max, f_mass, f_round, f_bad;
  __device__ __forceinline__ void row(int r, int k, double s, double sa) {
    const double x = acc[r];
    const double bb = b[r];
    const double p = p_scale * bb;
    const double res = bb - x + c * s + c * mx * p;
    r_out[r] = res;
    const double ar = fabs(res);
    if (!isfinite(res)) f_bad += 1.0;
    f_abs += ar;
    f_max = fmax(f_max, ar);
    f_mass += x;
    f_round += (static_cast<double>(k) + 5.0) * 0x1p-53 *
                   (fabs(bb) + fabs(x) + c * sa + c * fabs(mx) * p) +
               c * p * nu * mxa;
  }
};

struct DirResidArgs {
  const int* rp;
  const int* ci;
  const WorkItem* items;
  const double* w;
  const double* acc;
  const double* b;
  double* r;
  const double* dx;
  const double* dxa;
  double c, nu;
  double* stat_slots;
  double* split_part;
  int* split_count;
  const int* split_nchunks;
  int xcd;
};

template <int NPT>
__global__ __launch_bounds__(kWG) void k_resid_dir(DirResidArgs a) {
  __shared__ double m_sh[2];
  if (threadIdx.x < 64) {
    const double m = slot_sum(a.dx), ma = slot_sum(a.dxa);
    if (threadIdx.x == 0) {
      m_sh[0] = m;
      m_sh[1] = ma;
    }
  }
  __syncthreads();
  const int lb = xcd_logical(blockIdx.x, gridDim.x, a.xcd);
  DirResidEpi epi{a.acc, a.b, a.r, a.c, m_sh[0], m_sh[1], 1.0 / (1.0 - a.c), a.nu,
                  0.0, 0.0, 0.0, 0.0, 0.0};
  spmv_item<double, NPT, true>(a.items[lb], a.rp, a.ci, a.w, a.split_part, a.split_count,
                               a.split_nchunks, epi);
  const double s_abs = block_sum256(epi.f_abs);
  const double s_max = block_max256(epi.f_max);
  const double s_mass = block_sum256(epi.f_mass);
  const double s_round = block_sum256(epi.f_round);
  const double s_bad = block_sum256(epi.f_bad);
  if (threadIdx.x == 0) {
    double* o = a.stat_slots + (size_t)(lb % kSlots) * kStat;
    atomic_add(&o[0], s_abs);
    atomic_max_nonneg(&o[1], s_max);
    atomic_add(&o[3], s_mass);
    atomic_add(&o[4], s_round);
    if (s_bad != 0.0) atomic_add(&o[5], s_bad);
  }
}

// Residual of a column-sliced directed plan: k_resid_sliced left per slice
// the partial sums of w and of |w| over each row's in-neighbours; add the
// eight pairs and run k_resid_dir's epilogue (same rounding allowance: the
// partial sums and this addition are one summation of the row's k terms).
struct DirResidCombineArgs {
  const double2* part;
  const int* rp;
  const double* acc;
  const double* b;
  double* r;
  const double* dx;
  const double* dxa;
  double c, nu;
  double* stat_slots;
  int n;
};

__global__ __launch_bounds__(kWG) void k_resid_combine_dir(DirResidCombineArgs a) {
  __shared__ double m_sh[2];
  if (threadIdx.x < 64) {
    const double m = slot_sum(a.dx), ma = slot_sum(a.dxa);
    if (threadIdx.x == 0) {
      m_sh[0] = m;
      m_sh[1] = ma;
    }
  }
  __syncthreads();
  DirResidEpi epi{a.acc, a.b, a.r, a.c, m_sh[0], m_sh[1], 1.0 / (1.0 - a.c), a.nu,
                  0.0, 0.0, 0.0, 0.0, 0.0};
  const size_t n = static_cast<size_t>(a.n);
  for (int u = blockIdx.x * kWG + threadIdx.x; u < a.n; u += gridDim.x * kWG) {
    double s = 0.0, sa = 0.0;
#pragma unroll
    for (int k = 0; k < kSlices; ++k) {
      const double2 q = a.part[k * n + u];
      s += q.x;
      sa += q.y;
    }
    epi.row(u, a.rp[u + 1] - a.rp[u], s, sa);
  }
  const double s_abs = block_sum256(epi.f_abs);
  const double s_max = block_max256(epi.f_max);
  const double s_mass = block_sum256(epi.f_mass);
  const double s_round = block_sum256(epi.f_round);
  const double s_bad = block_sum256(epi.f_bad);
  if (threadIdx.x == 0) {
    double* o = a.stat_slots + (size_t)(blockIdx.x % kSlots) * kStat;
    atomic_add(&o[0], s_abs);
    atomic_max_nonneg(&o[1], s_max);
    atomic_add(&o[3], s_mass);
    atomic_add(&o[4], s_round);
    if (s_bad != 0.0) atomic_add(&o[5], s_bad);
  }
}

__global__ __launch_bounds__(kWG) void k_finalize_dir(int n, const int* __restrict__ perm,
                                                      const double* __restrict__ acc,
                                                      double scale, double* __restrict__ x) {
  for (int u = blockIdx.x * kWG + threadIdx.x; u < n; u += gridDim.x * kWG)
    x[perm ? perm[u] : u] = scale * acc[u];
}

// Column-sliced step on a directed plan: k_term_sliced left the partial sums
// of z over each column slice in part[s][row]; add them in a fixed order and
// run the directed epilogue.
struct DirCombineArgs {
  const float* part;
  const int* dout;
  const double* b;
  const double* x0;
  double x0_scale;
  float* zn;
  double* acc;
  const double* dang_cur;
  double* dang_next;
  double* dang_clear;
  double c;
  double* cert;
  const int* done;
  int n;
};

__global__ __launch_bounds__(kWG) void k_combine_dir(DirCombineArgs a) {
  if (a.done != nullptr && *a.done) return;
  __shared__ double m_sh;
  if (threadIdx.x < 64) {
    const double m = slot_sum(a.dang_cur);
    if (threadIdx.x == 0) m_sh = m;
  }
  if (blockIdx.x == 0 && threadIdx.x < kSlots) a.dang_clear[threadIdx.x] = 0.0;
  __syncthreads();
  DirTermEpi epi{a.b, a.x0, a.dout, a.zn, a.acc, a.c, m_sh, 1.0 / (1.0 - a.c), a.x0_scale,
                 a.cert != nullptr, 0.0, 0.0};
  const size_t n = static_cast<size_t>(a.n);
  for (int u = blockIdx.x * kWG + threadIdx.x; u < a.n; u += gridDim.x * kWG) {
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kSlices; ++k) s += a.part[k * n + u];
    epi.row(u, 0, s, 0.f);
  }
  const double cs = block_sum256(epi.cert);
  const double ms = block_sum256(epi.mnext);
  if (threadIdx.x == 0) {
    if (a.cert != nullptr && cs != 0.0) atomic_add(&a.cert[blockIdx.x % kSlots], cs);
    if (ms != 0.0) atomic_add(&a.dang_next[blockIdx.x % kSlots], ms);
  }
}

}  // namespace

hipError_t init_w1(const cpaa_plan_s* pl, Workspace& ws, const double* src, double scale,
                   bool add, bool store_b, bool series, hipStream_t st) {
  if (pl->fp64)
    hipLaunchKernelGGL(k_init_w1<double>, dim3(elem_grid(pl->n)), dim3(kWG), 0, st, pl->n,
                       pl->d_rp_w1, src == ws.r ? nullptr : pl->d_perm, src, scale, add ? 1 : 0,
                       store_b ? 1 : 0, series ? 1 : 0, series_a0(pl, ws), ws.b,
                       reinterpret_cast<double*>(ws.z[0]), ws.acc, ws.stat_slots,
                       pl->deterministic ? ws.det_part : nullptr, ws.det_count);
  else
    hipLaunchKernelGGL(k_init_w1<float>, dim3(elem_grid(pl->n)), dim3(kWG), 0, st, pl->n,
                       pl->d_rp_w1, src == ws.r ? nullptr : pl->d_perm, src, scale, add ? 1 : 0,
                       store_b ? 1 : 0, series ? 1 : 0, series_a0(pl, ws), ws.b, ws.z[0],
                       ws.acc, ws.stat_slots, pl->deterministic ? ws.det_part : nullptr,
                       ws.det_count);
  hipError_t e = hipGetLastError();
  // a caller's right-hand side: its dropped vertices join the statistics
  if (e == hipSuccess && store_b && src != ws.r) e = dropped_stats(pl, ws, src, st);
  return e;
}

hipError_t load_x0_w1(const cpaa_plan_s* pl, Workspace& ws, const double* x0, hipStream_t st) {
  hipLaunchKernelGGL(k_load_x0_w1, dim3(elem_grid(pl->n)), dim3(kWG), 0, st, pl->n,
                     pl->d_rp_w1, pl->d_perm, x0, ws.acc, ws.stat_slots);
  return hipGetLastError();
}

namespace {

template <typename V>
SlicedArgsT<V> sliced_args(const cpaa_plan_s* pl, const V* x, V* part, V* split_part,
                           int* split_count, const int* done) {
  SlicedArgsT<V> s;
  s.entries = pl->slc.d_entries;
  s.items = pl->slc.d_items;
  s.rp = pl->d_rp_w1;
  s.zc = x;
  s.part = part;
  s.done = done;
  s.split_part = split_part;
  s.split_count = split_count;
  s.split_nchunks = pl->slc.d_split_nchunks;
  s.n = pl->n;
  for (int i = 0; i <= kSlices; ++i) {
    s.item_off[i] = pl->slc.item_off[i];
    s.slice_off[i] = pl->slc.slice_off[i];
  }
  return s;
}

// Pass 1 of a column-sliced term: partial sums of z_cur per column slice into ws.part.
void sliced_pass(const cpaa_plan_s* pl, Workspace& ws, int cur, const int* done, hipStream_t st) {
  const SlicedArgs s = sliced_args<float>(pl, ws.z[cur], ws.part, ws.split_f, ws.split_count,
                                          done);
  const dim3 grid(kSlices * pl->slc.max_items);
  if (pl->slc.row_bits == kSliceRowBitsMax)
    hipLaunchKernelGGL((k_term_sliced<kSliceNpt, kSliceRowBitsMax>), grid, dim3(kWG), 0, st, s);
  else
    hipLaunchKernelGGL((k_term_sliced<kSliceNpt, 11>), grid, dim3(kWG), 0, st, s);
}

// Pass 1 of a hub-sliced term with launch shape cfg: partial sums of z_cur
// into ws.part.
template <typename V>
HubArgsT<V> hub_args(const cpaa_plan_s* pl, const V* x, V* part, V* chunk_val, int* long_cnt,
                     const int* done) {
  const HubMap& hm = pl->hub;
  HubArgsT<V> h;
  h.entries = hm.d_entries;
  h.items = hm.d_items;
  h.zc = x;
  h.part = part;
  h.done = done;
  h.chunk_val = chunk_val;
  h.long_cnt = long_cnt;
  h.chunk_long = hm.d_chunk_long;
  h.long_first = hm.d_long_first;
  h.long_nch = hm.d_long_nch;
  h.long_out = hm.d_long_out;
  for (int i = 0; i <= kSlices; ++i) {
    h.item_off[i] = hm.item_off[i];
    h.slice_off[i] = pl->slc.slice_off[i];
    h.pofs[i] = hm.pofs[i];
  }
  return h;
}

void hub_pass(const cpaa_plan_s* pl, Workspace& ws, int cur, const int* done, int cfg,
              hipStream_t st) {
  const HubArgs h = hub_args<float>(pl, ws.z[cur], ws.part, ws.chunk_val, ws.long_cnt, done);
  const dim3 grid(kSlices * pl->hub.groups[cfg]);
#define CPAA_HUB_LAUNCH(K)                                                            \
  hipLaunchKernelGGL((k_term_hub<kHubShapes[K].waves, kHubShapes[K].hub>), grid,      \
                     dim3(kHubShapes[K].waves * 64), 0, st, h)
  switch (cfg) {
    case 1: CPAA_HUB_LAUNCH(1); break;
    case 2: CPAA_HUB_LAUNCH(2); break;
    case 3: CPAA_HUB_LAUNCH(3); break;
    default: CPAA_HUB_LAUNCH(0); break;
  }
#undef CPAA_HUB_LAUNCH
}

}  // namespace

hipError_t term_w1(const cpaa_plan_s* pl, Workspace& ws, int cur, int prev, int next, bool first,
                   const AccUpdate& au, double* cert_slot, const int* done, hipStream_t st) {
  const TermShape sh = term_shape(pl, ws, first);
  if (pl->sliced && pl->hub.built) {
    hub_pass(pl, ws, cur, done, pl->hub.cfg, st);
    HubCombineArgs c;
    c.det_part = pl->deterministic ? ws.det_part : nullptr;
    c.det_count = ws.det_count;
    c.rp = pl->d_rp_w1;
    c.mask = pl->hub.d_mask;
    c.base = pl->hub.d_base;
    c.part = ws.part;
    for (int i = 0; i < kSlices; ++i) c.pofs[i] = pl->hub.pofs[i];
    c.zc = ws.z[cur];
    c.zp = first ? (sh.zp_is_cur ? ws.z[cur] : nullptr) : ws.z[prev];
    c.zn = ws.z[next];
    c.acc = ws.acc;
    c.alpha = sh.alpha;
    c.gamma_c = sh.gamma_c;
    c.gamma = sh.gamma;
    c.au = au;
    c.beta = sh.beta;
    c.cert = cert_slot;
    c.done = done;
    c.n = pl->n;
    hipLaunchKernelGGL(k_combine_hub, dim3((pl->n + kWG - 1) / kWG), dim3(kWG), 0, st, c);
    return hipGetLastError();
  }
  if (pl->sliced) {
    sliced_pass(pl, ws, cur, done, st);
    CombineArgs c;
    c.rp = pl->d_rp_w1;
    c.part = ws.part;
    c.zc = ws.z[cur];
    c.zp = first ? (sh.zp_is_cur ? ws.z[cur] : nullptr) : ws.z[prev];
    c.zn = ws.z[next];
    c.acc = ws.acc;
    c.alpha = sh.alpha;
    c.gamma_c = sh.gamma_c;
    c.gamma = sh.gamma;
    c.au = au;
    c.beta = sh.beta;
    c.cert = cert_slot;
    c.done = done;
    c.n = pl->n;
    hipLaunchKernelGGL(k_combine_w1, dim3(elem_grid(pl->n)), dim3(kWG), 0, st, c);
    return hipGetLastError();
  }
  if (pl->fp64) {
    // FP64 recurrence (debug option): the same row-order kernel in double
    double* const* zd = reinterpret_cast<double* const*>(ws.z);
    TermArgsT<double> a;
    a.rp = pl->d_rp_w1;
    a.ci = pl->d_ci_w1;
    a.items = pl->d_items;
    a.zc = zd[cur];
    a.zp = first ? (sh.zp_is_cur ? zd[cur] : nullptr) : zd[prev];
    a.zn = zd[next];
    a.acc = ws.acc;
    a.alpha = sh.alpha_d;
    a.gamma_c = sh.gamma_c_d;
    a.gamma = sh.gamma_d;
    a.au = au;
    a.beta = sh.beta;
    a.cert = cert_slot;
    a.done = done;
    a.split_part = ws.split_d;
    a.split_count = ws.split_count;
    a.split_nchunks = pl->d_split_nchunks;
    a.xcd = pl->xcd_remap;
    const dim3 grid(pl->n_items);
    switch (pl->npt) {
      case 4: hipLaunchKernelGGL((k_term_w1<4, double>), grid, dim3(kWG), 0, st, a); break;
      case 16: hipLaunchKernelGGL((k_term_w1<16, double>), grid, dim3(kWG), 0, st, a); break;
      case 32: hipLaunchKernelGGL((k_term_w1<32, double>), grid, dim3(kWG), 0, st, a); break;
      default: hipLaunchKernelGGL((k_term_w1<8, double>), grid, dim3(kWG), 0, st, a); break;
    }
    return hipGetLastError();
  }
  TermArgsT<float> a;
  a.rp = pl->d_rp_w1;
  a.ci = pl->d_ci_w1;
  a.items = pl->d_items;
  a.zc = ws.z[cur];
  a.zp = first ? (sh.zp_is_cur ? ws.z[cur] : nullptr) : ws.z[prev];
  a.zn = ws.z[next];
  a.acc = ws.acc;
  a.alpha = sh.alpha;
  a.gamma_c = sh.gamma_c;
  a.gamma = sh.gamma;
  a.au = au;
  a.beta = sh.beta;
  a.cert = cert_slot;
  a.done = done;
  a.split_part = ws.split_f;
  a.split_count = ws.split_count;
  a.split_nchunks = pl->d_split_nchunks;
  a.xcd = pl->xcd_remap;
  const dim3 grid(pl->n_items);
  switch (pl->npt) {
    case 4: hipLaunchKernelGGL((k_term_w1<4, float>), grid, dim3(kWG), 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_term_w1<16, float>), grid, dim3(kWG), 0, st, a); break;
    case 32: hipLaunchKernelGGL((k_term_w1<32, float>), grid, dim3(kWG), 0, st, a); break;
    default: hipLaunchKernelGGL((k_term_w1<8, float>), grid, dim3(kWG), 0, st, a); break;
  }
  return hipGetLastError();
}

hipError_t residual_w1(const cpaa_plan_s* pl, Workspace& ws, hipStream_t st, double* x,
                       bool* wrote_x) {
  if (wrote_x != nullptr) *wrote_x = false;
  if (pl->sliced && pl->hub.built && ws.part64 != nullptr) {
    // hub-sliced plans: FP64 partial sums of acc per slice on the term's map,
    // then the residual and its statistics per row
    const HubArgsT<double> h =
        hub_args<double>(pl, ws.acc, ws.part64, ws.chunk64, ws.long_cnt, nullptr);
    hipLaunchKernelGGL((k_term_hub<kHubResidShape.waves, kHubResidShape.hub, double>),
                       dim3(kSlices * pl->hub.groups_resid), dim3(kHubResidShape.waves * 64), 0,
                       st, h);
    ResidHubArgs r;
    r.rp = pl->d_rp_w1;
    r.mask = pl->hub.d_mask;
    r.base = pl->hub.d_base;
    r.part = ws.part64;
    for (int i = 0; i < kSlices; ++i) r.pofs[i] = pl->hub.pofs[i];
    r.acc = ws.acc;
    r.b = ws.b;
    r.wround = pl->hub.d_wround;
    r.r = ws.r;
    r.perm = pl->d_perm;
    r.x = pl->d_perm != nullptr ? x : nullptr;
    if (wrote_x != nullptr) *wrote_x = r.x != nullptr;
    r.c = pl->c;
    r.stat_slots = ws.stat_slots + (size_t)kSlots * ws.cols * kStat;   // residual phase
    r.det_part = pl->deterministic ? ws.det_part : nullptr;
    r.det_count = ws.det_count;
    r.n = pl->n;
    hipLaunchKernelGGL(k_resid_hub, dim3((pl->n + kWG - 1) / kWG), dim3(kWG), 0, st, r);
    return hipGetLastError();
  }
  ResidArgs a;
  a.rp = pl->d_rp_w1;
  a.ci = pl->d_ci_w1;
  a.items = pl->d_items;
  a.acc = ws.acc;
  a.b = ws.b;
  a.r = ws.r;
  a.c = pl->c;
  a.stat_slots = ws.stat_slots + (size_t)kSlots * ws.cols * kStat;   // residual phase
  a.split_part = ws.split_d;
  a.split_count = ws.split_count;
  a.split_nchunks = pl->d_split_nchunks;
  a.xcd = pl->xcd_remap;
  a.det_part = pl->deterministic ? ws.det_part : nullptr;
  a.det_count = ws.det_count;
  a.det_chunk = ws.det_chunk;
  a.max_chunks = ws.det_max_chunks;
  a.det_defer = ws.det_defer;
  a.n_split = pl->n_split_rows;
  const dim3 grid(pl->n_items);
  switch (pl->npt) {
    case 4: hipLaunchKernelGGL(k_resid_w1<4>, grid, dim3(kWG), 0, st, a); break;
    case 16: hipLaunchKernelGGL(k_resid_w1<16>, grid, dim3(kWG), 0, st, a); break;
    case 32: hipLaunchKernelGGL(k_resid_w1<32>, grid, dim3(kWG), 0, st, a); break;
    default: hipLaunchKernelGGL(k_resid_w1<8>, grid, dim3(kWG), 0, st, a); break;
  }
  return hipGetLastError();
}

namespace {

// One workgroup, a fixed summation order: the dropped vertices' p into the
// statistics of the right-hand side (so the whole p is validated).
__global__ __launch_bounds__(kWG) void k_dropped_stats(int nd, const int* __restrict__ dropped,
                                                       const double* __restrict__ src,
                                                       double* __restrict__ stat) {
  double sum = 0.0, neg = 0.0, bad = 0.0;
  for (int i = threadIdx.x; i < nd; i += kWG) {
    const double p = src[dropped[i]];
    sum += p;
    neg += p < 0.0 ? 1.0 : 0.0;
    bad += isfinite(p) ? 0.0 : 1.0;
  }
  sum = block_sum256(sum);
  neg = block_sum256(neg);
  bad = block_sum256(bad);
  if (threadIdx.x == 0) {
    atomic_add(&stat[0], sum);
    atomic_add(&stat[3], sum);
    if (neg != 0.0) atomic_add(&stat[4], neg);
    if (bad != 0.0) atomic_add(&stat[5], bad);
  }
}

__global__ __launch_bounds__(kWG) void k_dropped_out(int nd, const int* __restrict__ dropped,
                                                     const double* __restrict__ src, double scale,
                                                     double* __restrict__ x) {
  for (int i = blockIdx.x * kWG + threadIdx.x; i < nd; i += gridDim.x * kWG)
    x[dropped[i]] = scale * src[dropped[i]];
}

}  // namespace

hipError_t dropped_stats(const cpaa_plan_s* pl, Workspace& ws, const double* src,
                         hipStream_t st) {
  if (pl->n_drop == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dropped_stats, dim3(1), dim3(kWG), 0, st, pl->n_drop, pl->d_dropped, src,
                     ws.stat_slots);
  return hipGetLastError();
}

hipError_t dropped_out(const cpaa_plan_s* pl, const double* src, double scale, double* x,
                       hipStream_t st) {
  if (pl->n_drop == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dropped_out, dim3(elem_grid(pl->n_drop)), dim3(kWG), 0, st, pl->n_drop,
                     pl->d_dropped, src, scale, x);
  return hipGetLastError();
}

hipError_t finalize_w1(const cpaa_plan_s* pl, Workspace& ws, double* x, double scale,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_w1, dim3(elem_grid(pl->n)), dim3(kWG), 0, st, pl->n,
                     pl->d_rp_w1, pl->d_perm, ws.acc, scale, x);
  return hipGetLastError();
}

hipError_t init_dir(const cpaa_plan_s* pl, Workspace& ws, const double* src, double scale,
                    bool add, bool store_b, hipStream_t st) {
  hipLaunchKernelGGL(k_init_dir, dim3(elem_grid(pl->n)), dim3(kWG), 0, st, pl->n, pl->d_dout,
                     src == ws.r ? nullptr : pl->d_perm, src, scale, 1.0 - pl->c, add ? 1 : 0,
                     store_b ? 1 : 0, ws.b, ws.z[0], ws.acc, ws.dang, ws.stat_slots);
  return hipGetLastError();
}

hipError_t term_dir(const cpaa_plan_s* pl, Workspace& ws, int cur, int prev, int next, bool first,
                    const AccUpdate&, double* cert_slot, const int* done, hipStream_t st) {
  // every launch adds its increment to acc (x-space), so any stop leaves
  // acc = x_{k+1}; grouped updates do not apply here
  if (pl->sliced) {
    sliced_pass(pl, ws, cur, done, st);
    DirCombineArgs c;
    c.part = ws.part;
    c.dout = pl->d_dout;
    c.b = ws.b;
    c.x0 = first ? ws.dir_x0 : nullptr;
    c.x0_scale = ws.dir_x0_scale;
    c.zn = ws.z[next];
    c.acc = ws.acc;
    c.dang_cur = ws.dang + (size_t)cur * kSlots;
    c.dang_next = ws.dang + (size_t)next * kSlots;
    c.dang_clear = ws.dang + (size_t)prev * kSlots;
    c.c = pl->c;
    c.cert = cert_slot;
    c.done = done;
    c.n = pl->n;
    hipLaunchKernelGGL(k_combine_dir, dim3(elem_grid(pl->n)), dim3(kWG), 0, st, c);
    return hipGetLastError();
  }
  DirArgs a;
  a.rp = pl->d_rp_w1;
  a.ci = pl->d_ci_w1;
  a.items = pl->d_items;
  a.dout = pl->d_dout;
  a.b = ws.b;
  a.x0 = first ? ws.dir_x0 : nullptr;
  a.x0_scale = ws.dir_x0_scale;
  a.zc = ws.z[cur];
  a.zn = ws.z[next];
  a.acc = ws.acc;
  a.dang_cur = ws.dang + (size_t)cur * kSlots;
  a.dang_next = ws.dang + (size_t)next * kSlots;
  a.dang_clear = ws.dang + (size_t)prev * kSlots;
  a.c = pl->c;
  a.cert = cert_slot;
  a.done = done;
  a.split_part = ws.split_f;
  a.split_count = ws.split_count;
  a.split_nchunks = pl->d_split_nchunks;
  a.xcd = pl->xcd_remap;
  const dim3 grid(pl->n_items);
  switch (pl->npt) {
    case 4: hipLaunchKernelGGL(k_term_dir<4>, grid, dim3(kWG), 0, st, a); break;
    case 16: hipLaunchKernelGGL(k_term_dir<16>, grid, dim3(kWG), 0, st, a); break;
    case 32: hipLaunchKernelGGL(k_term_dir<32>, grid, dim3(kWG), 0, st, a); break;
    default: hipLaunchKernelGGL(k_term_dir<8>, grid, dim3(kWG), 0, st, a); break;
  }
  return hipGetLastError();
}

hipError_t residual_dir(const cpaa_plan_s* pl, Workspace& ws, hipStream_t st) {
  double* dx = ws.dang + 3 * kSlots;
  double* dxa = ws.dang + 4 * kSlots;
  hipError_t e = fill_f64(dx, 0.0, 2 * kSlots, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dir_w, dim3(elem_grid(pl->n)), dim3(kWG), 0, st, pl->n, pl->d_dout, ws.acc,
                     ws.wdir, dx, dxa);
  const double nu = (static_cast<double>(pl->n) + 2.0) * 0x1p-53;
  double* stat = ws.stat_slots + (size_t)kSlots * ws.cols * kStat;   // residual phase
  if (pl->sliced) {
    // FP64 gathers per column slice (pairs of partials), then the combine pass
    const SlicedArgsT<double> s = sliced_args<double>(pl, ws.wdir, ws.part_d, ws.split_d,
                                                      ws.split_count, nullptr);
    const dim3 grid(kSlices * pl->slc.max_items);
    if (pl->slc.row_bits == kSliceRowBitsMax)
      hipLaunchKernelGGL((k_resid_sliced<kSliceNpt, kSliceRowBitsMax>), grid, dim3(kWG), 0, st, s);
    else
      hipLaunchKernelGGL((k_resid_sliced<kSliceNpt, 11>), grid, dim3(kWG), 0, st, s);
    DirResidCombineArgs c;
    c.part = reinterpret_cast<const double2*>(ws.part_d);
    c.rp = pl->d_rp_w1;
    c.acc = ws.acc;
    c.b = ws.b;
    c.r = ws.r;
    c.dx = dx;
    c.dxa = dxa;
    c.c = pl->c;
    c.nu = nu;
    c.stat_slots = stat;
    c.n = pl->n;
    hipLaunchKernelGGL(k_resid_combine_dir, dim3(elem_grid(pl->n)), dim3(kWG), 0, st, c);
    return hipGetLastError();
  }
  DirResidArgs a;
  a.rp = pl->d_rp_w1;
  a.ci = pl->d_ci_w1;
  a.items = pl->d_items;
  a.w = ws.wdir;
  a.acc = ws.acc;
  a.b = ws.b;
  a.r = ws.r;
  a.dx = dx;
  a.dxa = dxa;
  a.c = pl->c;
  a.nu = nu;
  a.stat_slots = stat;
  a.split_part = ws.split_d;
  a.split_count = ws.split_count;
  a.split_nchunks = pl->d_split_nchunks;
  a.xcd = pl->xcd_remap;
  const dim3 grid(pl->n_items);
  switch (pl->npt) {
    case 4: hipLaunchKernelGGL(k_resid_dir<4>, grid, dim3(kWG), 0, st, a); break;
    case 16: hipLaunchKernelGGL(k_resid_dir<16>, grid, dim3(kWG), 0, st, a); break;
    case 32: hipLaunchKernelGGL(k_resid_dir<32>, grid, dim3(kWG), 0, st, a); break;
    default: hipLaunchKernelGGL(k_resid_dir<8>, grid, dim3(kWG), 0, st, a); break;
  }
  return hipGetLastError();
}

hipError_t finalize_dir(const cpaa_plan_s* pl, Workspace& ws, double* x, double scale,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_dir, dim3(elem_grid(pl->n)), dim3(kWG), 0, st, pl->n, pl->d_perm,
                     ws.acc, scale, x);
  return hipGetLastError();
}

}  // namespace cpaa
