// Small kernels shared by every solve path: fills, reduction collapse and the
// per-term stopping check.
#include "device.h"
#include "internal.h"

namespace cpaa {
namespace {

__global__ __launch_bounds__(kWG) void k_fill_f64(double* p, double v, size_t count) {
  for (size_t i = (size_t)blockIdx.x * kWG + threadIdx.x; i < count; i += (size_t)gridDim.x * kWG)
    p[i] = v;
}

__global__ __launch_bounds__(kWG) void k_fill_i32(int* p, int v, size_t count) {
  for (size_t i = (size_t)blockIdx.x * kWG + threadIdx.x; i < count; i += (size_t)gridDim.x * kWG)
    p[i] = v;
}

// stat[ph][col][f] = reduce over slots s of stat_slots[ph][s][col][f]; field 1 is a max.
__global__ __launch_bounds__(kWG) void k_collapse(const double* __restrict__ slots,
                                                  double* __restrict__ out, int64_t cols) {
  const int64_t per_phase = cols * kStat;
  const int64_t total = 2 * per_phase;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kWG) {
    const int64_t ph = i / per_phase, rest = i - ph * per_phase;
    const int f = static_cast<int>(rest % kStat);
    const double* src = slots + ph * kSlots * per_phase + rest;
    double acc = 0.0;
    for (int s = 0; s < kSlots; ++s) {
      const double v = src[(int64_t)s * per_phase];
      acc = (f == 1) ? fmax(acc, v) : acc + v;
    }
    out[i] = acc;
  }
}

// One workgroup (64 threads) per tile.  Column j of tile t is certified at this
// term if scale * sum_s cert_slot[s][t*W + j] <= target; when every column of
// the tile is, the tile stops (done[t] = 1) and records the term count.
__global__ __launch_bounds__(64) void k_check(const double* __restrict__ cert_slot, int64_t cols,
                                              int W, double scale, double target, int term_index,
                                              int* __restrict__ done, int* __restrict__ terms,
                                              double* __restrict__ series_cert) {
  const int t = blockIdx.x;
  if (done[t]) return;
  bool ok = true;
  for (int j = threadIdx.x; j < W; j += 64) {
    const int64_t col = (int64_t)t * W + j;
    double s = 0.0;
    for (int k = 0; k < kSlots; ++k) s += cert_slot[(int64_t)k * cols + col];
    const double v = s * scale;
    series_cert[col] = v;
    ok = ok && (v <= target);
  }
  const bool all = __all(ok);
  if (threadIdx.x == 0 && all) {
    done[t] = 1;
    terms[t] = term_index;
  }
}

__global__ void k_init_done(int* __restrict__ done, const int* __restrict__ active, int tiles) {
  for (int t = threadIdx.x; t < tiles; t += blockDim.x) done[t] = active ? !active[t] : 0;
}

int grid_for(size_t count) {
  const size_t g = (count + kWG - 1) / kWG;
  return static_cast<int>(g < 4096 ? (g < 1 ? 1 : g) : 4096);
}

}  // namespace

hipError_t fill_f64(double* p, double v, size_t count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(count)), dim3(kWG), 0, st, p, v, count);
  return hipGetLastError();
}

hipError_t fill_i32(int* p, int v, size_t count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(count)), dim3(kWG), 0, st, p, v, count);
  return hipGetLastError();
}

hipError_t collapse_stats(Workspace& ws, hipStream_t st) {
  hipLaunchKernelGGL(k_collapse, dim3(grid_for(2 * ws.cols * kStat)), dim3(kWG), 0, st,
                     ws.stat_slots, ws.stat, ws.cols);
  return hipGetLastError();
}

hipError_t init_done(Workspace& ws, const int* active, hipStream_t st) {
  hipLaunchKernelGGL(k_init_done, dim3(1), dim3(kWG), 0, st, ws.done, active, ws.tiles);
  return hipGetLastError();
}

hipError_t check_series(const cpaa_plan_s* pl, Workspace& ws, const double* cert_slot,
                        double scale, double target, int term_index, hipStream_t st) {
  (void)pl;
  hipLaunchKernelGGL(k_check, dim3(ws.tiles), dim3(64), 0, st, cert_slot, ws.cols, ws.W, scale,
                     target, term_index, ws.done, ws.terms, ws.series_cert);
  return hipGetLastError();
}

}  // namespace cpaa
