// Solve orchestration: one series of Chebyshev terms, the FP64 residual check,
// correction series on the residual, warm starts and the report.
//
// A series on right-hand side b (Sec. 3 eq. 3.1 applied to b) runs
//   term 0 (init):  z_0 = D^{-1} b,  acc (+)= (c_0/2) z_0
//   term 1:         z_1 = D^{-1} A z_0,  acc += c_1 z_1
//   term k+1:       z_{k+1} = 2 D^{-1} A z_k - z_{k-1},  acc += c_{k+1} z_{k+1}
// so x = D acc.  Stopping: the identity
//   b - (I - cP) x_M = ((1+s)/s) beta^{M+1} (T_{M+1}(P) b - beta T_M(P) b)
// (derived from eq. 3.1 and the three-term recurrence, s = sqrt(1-c^2)) gives
// an in-loop bound ||x_M - x||_1 <= ||.||_1/(1-c) from the last two vectors;
// the kernel producing z_{M+1} accumulates sum_u d_u |z_{M+1}(u) - beta z_M(u)|
// and a one-workgroup check kernel raises a device-side stop flag, so later
// term kernels exit at once and the host never waits inside a series.  The
// cap on terms is the a-priori bound sqrt(vol) ||D^{-1/2} b||_2 sum_{k>M} c_k
// (P = D^{1/2} S D^{-1/2} with S symmetric, spectrum in [-1,1] by Lemma 2),
// and no check runs before eq. 4.1's mass error ERR_M (a lower bound on the
// L1 error of a probability right-hand side) is below the target.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"

namespace cpaa {

void free_workspace(Workspace& ws) {
  void* ptrs[] = {ws.z[0], ws.z[1], ws.z[2], ws.acc, ws.part, ws.chunk_val, ws.long_cnt,
                  ws.part64, ws.chunk64,
                  ws.det_part, ws.det_count, ws.det_chunk, ws.det_defer,
                  ws.dang, ws.wdir, ws.part_d,
                  ws.b, ws.r,
                  ws.slots, ws.stat_slots,
                  ws.stat, ws.done, ws.terms, ws.series_cert, ws.split_f, ws.split_d,
                  ws.split_count, ws.active, ws.plain, ws.col_scale};
  if (!ws.external) {
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    if (ws.host) (void)hipHostFree(ws.host);
    if (ws.poll_host) (void)hipHostFree(ws.poll_host);
  }
  ws = Workspace();
}

// Host mirror layout (pinned): stat[2][cols][kStat] | series_cert[cols] | col_scale[cols] |
// done[tiles] | terms[tiles] | active[tiles] | plain[cols]
static size_t host_mirror_bytes(int64_t cols, int tiles) {
  return (size_t)(2 * kStat + 2) * cols * sizeof(double) + (size_t)(3 * tiles + cols) * sizeof(int) +
         64;
}

// Device buffers of a workspace for W right-hand sides per tile, each taken
// from `alloc(void** p, size_t bytes)` (which returns false when it cannot);
// ws.W, ws.tiles, ws.cols and ws.vec_elems are set here.  Without `resid64`
// the FP64 partials of the hub-sliced residual are left out (the residual then
// runs in row order).
template <typename Alloc>
bool layout_workspace(const cpaa_plan_s* pl, Workspace& ws, int W, int tiles, Alloc alloc,
                      bool resid64 = true) {
  ws.W = W;
  ws.tiles = tiles;
  ws.cols = static_cast<int64_t>(tiles) * W;
  ws.vec_elems = static_cast<size_t>(pl->n) * ws.cols;
  // split-row partial sums: one set per tile (tiles run concurrently)
  const size_t nsplit = (size_t)std::max(
      W == 1 ? std::max(pl->max_split_rows, pl->slc.n_split_rows) : pl->n_tsplit_rows, 1);
  const size_t split_sets = (size_t)tiles;
  bool ok = true;
  // the FP64 recurrence (single-vector path only) keeps doubles in the z buffers
  const size_t zbytes = (W == 1 && pl->fp64) ? sizeof(double) : sizeof(float);
  for (int i = 0; i < 3; ++i) ok = ok && alloc((void**)&ws.z[i], ws.vec_elems * zbytes);
  ok = ok && alloc((void**)&ws.acc, ws.vec_elems * sizeof(double));
  if (W == 1 && pl->sliced && pl->hub.built) {
    ok = ok && alloc((void**)&ws.part, (size_t)pl->hub.pofs[kSlices] * sizeof(float));
    ok = ok && alloc((void**)&ws.chunk_val, (size_t)pl->hub.n_chunks * sizeof(float));
    ok = ok && alloc((void**)&ws.long_cnt, (size_t)pl->hub.n_long * sizeof(int));
    if (resid64) {
      ok = ok && alloc((void**)&ws.part64, (size_t)pl->hub.pofs[kSlices] * sizeof(double));
      ok = ok && alloc((void**)&ws.chunk64, (size_t)pl->hub.n_chunks * sizeof(double));
    }
  } else if (W == 1 && pl->sliced) {
    ok = ok && alloc((void**)&ws.part, (size_t)kSlices * pl->n * sizeof(float));
  }
  if (W == 1 && pl->deterministic) {
    // per-block partials of the largest grid that reduces: the combine pass
    // (one row per thread), the init kernel, the residual (one block per item)
    const size_t blocks = std::max<size_t>({(size_t)(pl->n + kWG - 1) / kWG, (size_t)8192,
                                            (size_t)std::max(pl->n_items, 1)});
    ws.det_max_chunks = pl->max_deg / (kWG * 4) + 2;   // chunks of 256 x 4 entries or more
    ok = ok && alloc((void**)&ws.det_part, 4 * blocks * sizeof(double));
    ok = ok && alloc((void**)&ws.det_count, sizeof(int));
    ok = ok && alloc((void**)&ws.det_chunk,
                     (size_t)std::max(pl->max_split_rows, 1) * ws.det_max_chunks * 2 *
                         sizeof(double));
    ok = ok && alloc((void**)&ws.det_defer,
                     (size_t)std::max(pl->max_split_rows, 1) * 3 * sizeof(double));
  }
  if (W == 1 && pl->directed) {
    ok = ok && alloc((void**)&ws.dang, (size_t)5 * kSlots * sizeof(double));
    ok = ok && alloc((void**)&ws.wdir, (size_t)pl->n * sizeof(double));
    if (pl->sliced)
      ok = ok && alloc((void**)&ws.part_d, (size_t)kSlices * pl->n * 2 * sizeof(double));
  }
  ok = ok && alloc((void**)&ws.b, ws.vec_elems * sizeof(double));
  ok = ok && alloc((void**)&ws.r, ws.vec_elems * sizeof(double));
  ok = ok && alloc((void**)&ws.slots, (size_t)(kMaxTerms + 2) * kSlots * ws.cols * sizeof(double));
  ok = ok && alloc((void**)&ws.stat_slots, (size_t)2 * kSlots * ws.cols * kStat * sizeof(double));
  ok = ok && alloc((void**)&ws.stat, (size_t)2 * ws.cols * kStat * sizeof(double));
  ok = ok && alloc((void**)&ws.done, (size_t)tiles * sizeof(int));
  ok = ok && alloc((void**)&ws.terms, (size_t)tiles * sizeof(int));
  ok = ok && alloc((void**)&ws.series_cert, (size_t)ws.cols * sizeof(double));
  ok = ok && alloc((void**)&ws.split_f, split_sets * nsplit * W * sizeof(float));
  ok = ok && alloc((void**)&ws.split_d, split_sets * nsplit * 2 * W * sizeof(double));
  ok = ok && alloc((void**)&ws.split_count, split_sets * nsplit * sizeof(int));
  ok = ok && alloc((void**)&ws.active, (size_t)tiles * sizeof(int));
  ok = ok && alloc((void**)&ws.plain, (size_t)ws.cols * sizeof(int));
  ok = ok && alloc((void**)&ws.col_scale, (size_t)ws.cols * sizeof(double));
  ws.split_elems = split_sets * nsplit;
  return ok;
}

// Buffers that must start at zero: split-row partials and arrival counters,
// long-row chunk sums and counters, the deterministic arrival counter (every
// protocol leaves them at zero again).  With fill kernels (`async`, for a
// caller that may not allocate or synchronise) or synchronous memsets.
static cpaa_status zero_workspace(Workspace& ws, const cpaa_plan_s* pl, bool async,
                                  hipStream_t st) {
  const size_t nsp = ws.split_elems;
  if (async) {
    CPAA_HIP(fill_i32(reinterpret_cast<int*>(ws.split_f), 0, nsp * ws.W, st));
    CPAA_HIP(fill_f64(ws.split_d, 0.0, nsp * 2 * ws.W, st));
    CPAA_HIP(fill_i32(ws.split_count, 0, nsp, st));
    if (ws.chunk_val)
      CPAA_HIP(fill_i32(reinterpret_cast<int*>(ws.chunk_val), 0, (size_t)pl->hub.n_chunks, st));
    if (ws.long_cnt) CPAA_HIP(fill_i32(ws.long_cnt, 0, (size_t)pl->hub.n_long, st));
    if (ws.chunk64) CPAA_HIP(fill_f64(ws.chunk64, 0.0, (size_t)pl->hub.n_chunks, st));
    if (ws.det_count) CPAA_HIP(fill_i32(ws.det_count, 0, 1, st));
    return CPAA_OK;
  }
  bool ok = hipMemset(ws.split_f, 0, nsp * ws.W * sizeof(float)) == hipSuccess &&
            hipMemset(ws.split_d, 0, nsp * 2 * ws.W * sizeof(double)) == hipSuccess &&
            hipMemset(ws.split_count, 0, nsp * sizeof(int)) == hipSuccess;
  if (ok && ws.chunk_val)
    ok = hipMemset(ws.chunk_val, 0, (size_t)std::max(pl->hub.n_chunks, 1) * sizeof(float)) ==
         hipSuccess;
  if (ok && ws.long_cnt)
    ok = hipMemset(ws.long_cnt, 0, (size_t)std::max(pl->hub.n_long, 1) * sizeof(int)) ==
         hipSuccess;
  if (ok && ws.chunk64)
    ok = hipMemset(ws.chunk64, 0, (size_t)std::max(pl->hub.n_chunks, 1) * sizeof(double)) ==
         hipSuccess;
  if (ok && ws.det_count) ok = hipMemset(ws.det_count, 0, sizeof(int)) == hipSuccess;
  if (ok) ok = hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    set_error("workspace initialisation failed");
    return CPAA_EDEVICE;
  }
  return CPAA_OK;
}

cpaa_status ensure_workspace(cpaa_plan_s* pl, Workspace& ws, int W, int tiles) {
  if (ws.W == W && ws.tiles == tiles && ws.z[0]) return CPAA_OK;
  free_workspace(ws);
  auto alloc = [&](void** p, size_t bytes) -> bool {
    if (bytes == 0) bytes = 8;
    if (hipMalloc(p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return false;
    }
    return true;
  };
  bool ok = layout_workspace(pl, ws, W, tiles, alloc);
  ws.host_bytes = host_mirror_bytes(ws.cols, tiles);
  if (ok && hipHostMalloc((void**)&ws.host, ws.host_bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    ws.host = nullptr;
    ok = false;
  }
  if (ok && hipHostMalloc((void**)&ws.poll_host, (size_t)2 * tiles * sizeof(int),
                          hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    ws.poll_host = nullptr;
    ok = false;
  }
  if (!ok) {
    const int64_t cols = ws.cols;
    free_workspace(ws);
    set_error("workspace allocation failed (n = " + std::to_string(pl->n) +
              ", columns = " + std::to_string(static_cast<long long>(cols)) + ")");
    return CPAA_ENOMEM;
  }
  const cpaa_status s = zero_workspace(ws, pl, false, nullptr);
  if (s != CPAA_OK) free_workspace(ws);
  return s;
}

double series_tail(const cpaa_plan_s* pl, int M) {
  // sum_{k>M} c_k = (2/(A s)) beta^{M+1} / (1 - beta)
  return 2.0 / (pl->cheb_A * pl->s) * std::pow(pl->beta, M + 1) / (1.0 - pl->beta);
}

int apriori_terms(const cpaa_plan_s* pl, double q, double target) {
  // q = sum_u b_u^2 / d_u = ||D^{-1/2} b||_2^2
  const int cap = pl->opts.k_max > 0 ? std::min(pl->opts.k_max, kMaxTerms) : kMaxTerms;
  const double scale = std::sqrt(pl->vol) * std::sqrt(std::max(q, 0.0));
  if (!(scale > 0.0)) return 0;
  for (int M = 0; M <= cap; ++M)
    if (scale * series_tail(pl, M) <= target) return M;
  return cap;
}

int mass_rule_terms(const cpaa_plan_s* pl, double target) {
  // eq. 4.1: ERR_M = 2 beta^{M+1} / (1 + beta)
  for (int M = 0; M < kMaxTerms; ++M)
    if (2.0 * std::pow(pl->beta, M + 1) / (1.0 + pl->beta) <= target) return M;
  return kMaxTerms;
}

// Launches a series runs at most.  Chebyshev: the a-priori bound's term count
// for ||x_M - x*||_1 <= target (q = ||D^{-1/2}b||_2^2), x* the solution for
// the right-hand side b.  Power method: until its own certificate must pass,
// ||delta_M||_1 / (1-c) <= target, where ||delta_M||_1 <= c^M ||delta_0||_1 and
// ||delta_0||_1 = c ||(P - I) x_0||_1 <= 2c ||b||_1 / (1-c) (x_0 = b/(1-c)); the
// check of x_M runs in launch M, so M + 1 launches.  (The residual bound can be
// 1/(1-c) looser than the error itself, e.g. on bipartite graphs, so a cap from
// the error's contraction alone can end the series before the check passes.)
int series_cap(const cpaa_plan_s* pl, const Workspace& ws, double q, double b_l1,
               double target) {
  if (ws.method != Method::kPower) return apriori_terms(pl, q, target);
  const int cap = pl->opts.k_max > 0 ? std::min(pl->opts.k_max, kMaxTerms) : kMaxTerms;
  const double c = pl->c;
  double e = 2.0 * c * std::max(b_l1, 0.0) / ((1.0 - c) * (1.0 - c));
  if (!(e > 0.0)) return 0;
  for (int M = 0; M < cap; ++M, e *= c)
    if (e <= target) return M + 1;
  return cap;
}

// First launch whose certificate is checked: for a Chebyshev series on
// b = (1-c)p eq. 4.1's term (no earlier stop is possible for a distribution
// p), else the first; the power method is checked from its first launch on.
int series_first_check(const cpaa_plan_s* pl, const Workspace& ws, double target, bool from_p) {
  if (ws.method == Method::kPower) return 0;
  return from_p ? mass_rule_terms(pl, target) : 1;
}

namespace {

// Device time of term launches, from HIP events on the solve's stream.
// mode 1: one pair of events around every term launch (each event adds about
// 10 us of idle time between launches on this device); mode 2: one pair around
// each series of back-to-back term launches, whose time includes what little
// idle time lies between its kernels.
struct TermTimer {
  cpaa_plan_s* pl;
  int mode;   // 0 off, 1 per term, 2 per series
  struct Rec {
    int ev;          // index of the first event of the pair
    int series;
    int term;        // index of the (first) term the bracketed launches produce
    int last;        // index of the last one
  };
  std::vector<Rec> recs;
  int used = 0;
  bool open = false;   // mode 2: a series bracket is open
  hipError_t new_pair(int series, int term, hipStream_t st) {
    while ((int)pl->ev_terms.size() < used + 2) {
      hipEvent_t e;
      hipError_t err = hipEventCreate(&e);
      if (err != hipSuccess) return err;
      pl->ev_terms.push_back(e);
    }
    recs.push_back({used, series, term, term});
    hipError_t err = hipEventRecord(pl->ev_terms[used], st);
    used += 2;
    return err;
  }
  hipError_t before(int series, int term, hipStream_t st) {
    if (mode == 0) return hipSuccess;
    if (mode == 2 && open) {
      recs.back().last = term;
      return hipSuccess;
    }
    open = mode == 2;
    return new_pair(series, term, st);
  }
  hipError_t after(hipStream_t st) {
    if (mode != 1) return hipSuccess;
    return hipEventRecord(pl->ev_terms[recs.back().ev + 1], st);
  }
  hipError_t end_series(hipStream_t st) {
    if (mode != 2 || !open) return hipSuccess;
    open = false;
    return hipEventRecord(pl->ev_terms[recs.back().ev + 1], st);
  }
  // device time of the launches that did work (term <= terms run by their
  // series) and their number; mode 2 brackets hold whole series, whose
  // launches past the stop return at once
  void total(const std::vector<int>& series_terms, double* ms, int64_t* launches) {
    *ms = 0.0;
    *launches = 0;
    for (const Rec& r : recs) {
      const int worked = std::min(r.last, series_terms[r.series]) - r.term + 1;
      if (worked <= 0) continue;
      float t = 0.f;
      if (hipEventElapsedTime(&t, pl->ev_terms[r.ev], pl->ev_terms[r.ev + 1]) == hipSuccess) {
        *ms += t;
        *launches += worked;
      }
    }
  }
};

using TermFn = hipError_t (*)(const cpaa_plan_s*, Workspace&, int, int, int, bool,
                              const AccUpdate&,
                              double*, const int*, hipStream_t);

// Accumulator updates of launches 0..k_cap-1 (launch k produces z_{k+1} and
// owes c_{k+1} z_{k+1}).  A launch may leave its term to a later launch of
// the same series, whose epilogue still holds z_{k-1} and z_k:
//  * before the first check (k + 1 < k_min) in groups of three: off, off, on
//    with c_{k-1}, c_k, c_{k+1}; no stop can happen inside such a group;
//  * otherwise in pairs: off, on with c_k, c_{k+1}.  The off launch follows an
//    on launch, so acc holds exactly x_k = sum_{i<=k} c_i z_i when the off
//    launch's check certifies x_k; if the series stops there, the pending
//    term (beyond the certified x_k) is dropped.
std::vector<AccUpdate> acc_schedule(const std::vector<double>& ck, int k_cap, int k_min) {
  std::vector<AccUpdate> plan(std::max(k_cap, 0), AccUpdate{0.0, 0.0, 0.0, 1});
  int k = 0;
  while (k < k_cap) {
    if (k + 1 < k_min && k + 2 < k_cap) {
      plan[k].on = 0;
      plan[k + 1].on = 0;
      plan[k + 2] = AccUpdate{ck[k + 1], ck[k + 2], ck[k + 3], 1};
      k += 3;
    } else if (k + 1 < k_cap) {
      plan[k].on = 0;
      plan[k + 1] = AccUpdate{0.0, ck[k + 1], ck[k + 2], 1};
      k += 2;
    } else {
      plan[k] = AccUpdate{0.0, 0.0, ck[k + 1], 1};
      k += 1;
    }
  }
  return plan;
}

// Launch terms 1..k_cap of a series whose init already ran.  Returns after
// enqueueing; the stop flag / term count live in ws.done / ws.terms.  With
// `active` (device [tiles]) only the active tiles run.
cpaa_status run_series(cpaa_plan_s* pl, Workspace& ws, TermFn term, int series_id, int k_cap,
                       int k_min, double target, TermTimer& timer, hipStream_t st,
                       const int* active = nullptr) {
  const int64_t cols = ws.cols;
  CPAA_HIP(fill_f64(ws.slots, 0.0, (size_t)(k_cap + 1) * kSlots * cols, st));
  CPAA_HIP(init_done(ws, active, st));
  CPAA_HIP(fill_i32(ws.terms, k_cap, ws.tiles, st));
  CPAA_HIP(fill_f64(ws.series_cert, -1.0, cols, st));
  const std::vector<AccUpdate> acc_plan = acc_schedule(series_coef(pl, ws), k_cap, k_min);
  // The power method's a-priori cap (from c^k alone) can run far past the stop,
  // so its launches are enqueued in chunks and the stop flags are read one chunk
  // behind (the GPU always has the next chunk queued).  A stop inside chunk j
  // is seen after chunk j + 1 is enqueued, so up to 2 kChunk - 1 launches past
  // the stop are issued; they return at once.
  constexpr int kChunk = 4;
  const bool poll = ws.method == Method::kPower && ws.poll_host != nullptr &&
                    pl->ev_poll[0] != nullptr && k_cap > 2 * kChunk;
  int chunk = 0;
  for (int k = 0; k < k_cap; ++k) {
    // this launch produces z_{k+1}; its certificate is that of x_k
    double* cert = (k >= k_min) ? ws.slots + (size_t)k * kSlots * cols : nullptr;
    const int* done = (active != nullptr || (k >= 1 && k - 1 >= k_min)) ? ws.done : nullptr;
    CPAA_HIP(timer.before(series_id, k + 1, st));
    CPAA_HIP(term(pl, ws, k % 3, (k + 2) % 3, (k + 1) % 3, k == 0, acc_plan[k], cert, done, st));
    CPAA_HIP(timer.after(st));
    if (cert) {
      const double scale = ws.method == Method::kPower
                               ? 1.0 / ((1.0 - pl->c) * (1.0 - pl->c))
                               : (1.0 + pl->s) / pl->s * std::pow(pl->beta, k + 1) / (1.0 - pl->c);
      CPAA_HIP(check_series(pl, ws, cert, scale, target, k + 1, st));
    }
    if (poll && (k + 1) % kChunk == 0 && k + 1 < k_cap) {
      int* flags = ws.poll_host + (size_t)(chunk % 2) * ws.tiles;
      CPAA_HIP(hipMemcpyAsync(flags, ws.done, ws.tiles * sizeof(int), hipMemcpyDeviceToHost, st));
      CPAA_HIP(hipEventRecord(pl->ev_poll[chunk % 2], st));
      if (chunk > 0) {
        CPAA_HIP(hipEventSynchronize(pl->ev_poll[(chunk - 1) % 2]));
        const int* prev = ws.poll_host + (size_t)((chunk - 1) % 2) * ws.tiles;
        bool all = true;
        for (int t = 0; t < ws.tiles && all; ++t) all = prev[t] != 0;
        if (all) break;
      }
      ++chunk;
    }
  }
  CPAA_HIP(timer.end_series(st));
  return CPAA_OK;
}

// Time `reps` term launches (first term included) of the current work map on
// the workspace's current z_0; returns milliseconds per launch.  The probes
// write z and acc, so callers restart the series afterwards.
float time_terms(cpaa_plan_s* pl, Workspace& ws, TermFn term, int reps, hipStream_t st,
                 hipError_t* err) {
  *err = hipEventRecord(pl->ev_begin, st);
  for (int k = 0; k < reps && *err == hipSuccess; ++k)
    *err = term(pl, ws, k % 3, (k + 2) % 3, (k + 1) % 3, k == 0, AccUpdate{0.0, 0.0, 0.0, 1},
                nullptr, nullptr, st);
  if (*err == hipSuccess) *err = hipEventRecord(pl->ev_end, st);
  if (*err == hipSuccess) *err = hipEventSynchronize(pl->ev_end);
  float ms = 0.f;
  if (*err == hipSuccess) *err = hipEventElapsedTime(&ms, pl->ev_begin, pl->ev_end);
  return ms / reps;
}

struct HostView {
  double* stat;
  double* series_cert;
  double* col_scale;
  int* done;
  int* terms;
  int* active;
  int* plain;
};

HostView host_view(Workspace& ws) {
  HostView v;
  v.stat = ws.host;
  v.series_cert = v.stat + 2 * ws.cols * kStat;
  v.col_scale = v.series_cert + ws.cols;
  v.done = reinterpret_cast<int*>(v.col_scale + ws.cols);
  v.terms = v.done + ws.tiles;
  v.active = v.terms + ws.tiles;
  v.plain = v.active + ws.tiles;
  return v;
}

cpaa_status read_back(Workspace& ws, hipStream_t st) {
  HostView v = host_view(ws);
  CPAA_HIP(collapse_stats(ws, st));
  CPAA_HIP(hipMemcpyAsync(v.stat, ws.stat, 2 * ws.cols * kStat * sizeof(double),
                          hipMemcpyDeviceToHost, st));
  CPAA_HIP(hipMemcpyAsync(v.series_cert, ws.series_cert, ws.cols * sizeof(double),
                          hipMemcpyDeviceToHost, st));
  CPAA_HIP(hipMemcpyAsync(v.done, ws.done, ws.tiles * sizeof(int), hipMemcpyDeviceToHost, st));
  CPAA_HIP(hipMemcpyAsync(v.terms, ws.terms, ws.tiles * sizeof(int), hipMemcpyDeviceToHost, st));
  CPAA_HIP(hipStreamSynchronize(st));
  return CPAA_OK;
}

inline double stat_at(Workspace& ws, int phase, int64_t col, int f) {
  return host_view(ws).stat[(phase * ws.cols + col) * kStat + f];
}

cpaa_status check_p_stats(Workspace& ws, int64_t col) {
  const double sum = stat_at(ws, 0, col, 0);
  const double neg = stat_at(ws, 0, col, 4);
  const double bad = stat_at(ws, 0, col, 5);
  if (bad != 0.0 || !std::isfinite(sum)) {
    set_error("personalization vector has non-finite entries");
    return CPAA_EINVAL;
  }
  if (neg != 0.0) {
    set_error("personalization vector has negative entries");
    return CPAA_EINVAL;
  }
  if (std::fabs(sum - 1.0) > 1e-9) {
    set_error("personalization vector must sum to 1 (sum = " + std::to_string(sum) + ")");
    return CPAA_EINVAL;
  }
  return CPAA_OK;
}

// ||x - (I-cP)^{-1} b||_1 <= ||r||_1 / (1-c) for column-stochastic P.  The
// computed ||r||_1 is inflated by the kernels' bound on the rounding of r
// (round), by the rounding of x = D acc (u * mass) and by the rounding of the
// n-term sum itself, so the reported figure bounds the error of the x returned.
double rigorous_bound(const cpaa_plan_s* pl, double resid_l1, double round, double mass) {
  const double u = 0x1p-53;
  const double sum_err = 1.0 + 2.0 * u * static_cast<double>(pl->n);
  return (resid_l1 * sum_err + round) / (1.0 - pl->c) + u * std::fabs(mass);
}

// RAII device buffers for host-pointer I/O
struct TempDev {
  void* p = nullptr;
  ~TempDev() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace
}  // namespace cpaa

using namespace cpaa;

namespace {

cpaa_status solve_directed(cpaa_plan_t pl, const double* p, double tol, double* x,
                           cpaa_report* rep, void* stream);

cpaa_status solve_single(cpaa_plan_t pl, const double* p, double tol, const double* x0, double* x,
                         cpaa_report* rep, void* stream, Method method,
                         Workspace* ext = nullptr);

// Batched solves of plans whose options live on the single-vector path only
// (fp64_recurrence, deterministic): one column after another.
cpaa_status solve_columns(cpaa_plan_t pl, int32_t B, const double* P, int64_t ldp, double tol,
                          const double* X0, int64_t ldx0, double* X, int64_t ldx,
                          cpaa_report* reps, void* stream, Method method) {
  bool all_ok = true;
  for (int32_t j = 0; j < B; ++j) {
    cpaa_report R;
    std::memset(&R, 0, sizeof(R));
    const cpaa_status s = solve_single(pl, P + (size_t)j * ldp, tol,
                                       X0 ? X0 + (size_t)j * ldx0 : nullptr,
                                       X + (size_t)j * ldx, &R, stream, method);
    if (s != CPAA_OK && s != CPAA_ENOCONV) return s;
    all_ok = all_ok && s == CPAA_OK;
    if (reps) reps[j] = R;
  }
  if (!all_ok) {
    set_error("tolerance not certified for every column");
    return CPAA_ENOCONV;
  }
  set_error("");
  return CPAA_OK;
}

// Batched solves of a directed plan: the power method, one column after
// another through the single-vector path (no tiled directed kernel).
cpaa_status solve_directed_columns(cpaa_plan_t pl, int32_t B, const double* P, int64_t ldp,
                                   double tol, double* X, int64_t ldx, cpaa_report* reps,
                                   void* stream) {
  bool all_ok = true;
  for (int32_t j = 0; j < B; ++j) {
    cpaa_report R;
    std::memset(&R, 0, sizeof(R));
    const cpaa_status s = solve_directed(pl, P + (size_t)j * ldp, tol, X + (size_t)j * ldx, &R,
                                         stream);
    if (s != CPAA_OK && s != CPAA_ENOCONV) return s;
    all_ok = all_ok && s == CPAA_OK;
    if (reps) reps[j] = R;
  }
  if (!all_ok) {
    set_error("tolerance not certified for every column");
    return CPAA_ENOCONV;
  }
  set_error("");
  return CPAA_OK;
}

// ext: a workspace the caller has laid out (the no-allocation entry point);
// the solve then allocates nothing and records no timing events.
cpaa_status solve_single(cpaa_plan_t pl, const double* p, double tol, const double* x0, double* x,
                         cpaa_report* rep, void* stream, Method method, Workspace* ext) {
  set_error("");
  if (pl && pl->directed) {
    // CPAA's expansion needs the real spectrum of an undirected graph, so every
    // solve of a directed plan runs the power method (report.method = 1)
    if (x0) {
      set_error("a directed plan has no warm start (x0 must be NULL)");
      return CPAA_EINVAL;
    }
    return solve_directed(pl, p, tol, x, rep, stream);
  }
  if (!pl || !p || !x) {
    set_error("cpaa_solve: null argument");
    return CPAA_EINVAL;
  }
  if (!(tol > 0.0) || !std::isfinite(tol)) {
    set_error("tol must be positive and finite");
    return CPAA_EINVAL;
  }
  if (pl->num_graphs > 1) {
    set_error("block-diagonal plans are solved with cpaa_solve_graphs");
    return CPAA_EINVAL;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  cpaa_status s = ext ? CPAA_OK : ensure_workspace(pl, pl->ws1, 1, 1);
  if (s != CPAA_OK) return s;
  Workspace& ws = ext ? *ext : pl->ws1;
  ws.method = method;
  const int n = pl->n;
  const double c = pl->c;

  TempDev tp, tx0, tx;
  const double* dp = p;
  const double* dx0 = x0;
  double* dx = x;
  const size_t n_io = static_cast<size_t>(pl->n_caller);   // p, x0, x: the caller's vertices
  if (!pl->opts.io_device) {
    if (hipMalloc(&tp.p, n_io * sizeof(double)) != hipSuccess ||
        hipMalloc(&tx.p, n_io * sizeof(double)) != hipSuccess ||
        (x0 && hipMalloc(&tx0.p, n_io * sizeof(double)) != hipSuccess)) {
      (void)hipGetLastError();
      set_error("device allocation for host I/O failed");
      return CPAA_ENOMEM;
    }
    CPAA_HIP(hipMemcpyAsync(tp.p, p, n_io * sizeof(double), hipMemcpyHostToDevice, st));
    if (x0) CPAA_HIP(hipMemcpyAsync(tx0.p, x0, n_io * sizeof(double), hipMemcpyHostToDevice, st));
    dp = static_cast<const double*>(tp.p);
    dx0 = x0 ? static_cast<const double*>(tx0.p) : nullptr;
    dx = static_cast<double*>(tx.p);
  }

  TermTimer timer{pl, ext == nullptr ? pl->opts.time_kernels : 0};
  std::vector<int> series_terms;
  cpaa_report R;
  std::memset(&R, 0, sizeof(R));
  R.method = method == Method::kPower ? 1 : 0;
  CPAA_HIP(hipEventRecord(pl->ev_begin, st));
  CPAA_HIP(fill_f64(ws.stat_slots, 0.0, (size_t)2 * kSlots * ws.cols * kStat, st));

  bool warm = dx0 != nullptr;
  bool p_checked = false;
  double q0 = 0.0;    // ||D^{-1/2} b'||^2 of the first series' right-hand side
  double b0_l1 = 0.0; // ||b'||_1 of the same
  bool skip_series = false;
  if (warm) {
    CPAA_HIP(load_x0_w1(pl, ws, dx0, st));
    // b = (1-c) p only (no series start), then r0 = b - (I - cP) x0
    CPAA_HIP(init_w1(pl, ws, dp, 1.0 - c, false, true, false, st));
    CPAA_HIP(residual_w1(pl, ws, st));
    if ((s = read_back(ws, st)) != CPAA_OK) return s;
    if ((s = check_p_stats(ws, 0)) != CPAA_OK) return s;
    p_checked = true;
    const double r0 = stat_at(ws, 1, 0, 0);
    const double bnorm = (1.0 - c) * stat_at(ws, 0, 0, 0);
    const bool finite = stat_at(ws, 0, 0, 1) == 0.0 && stat_at(ws, 1, 0, 5) == 0.0 &&
                        std::isfinite(r0);
    if (!finite || !(r0 < bnorm)) {
      warm = false;
      R.fallback_used = 1;
    } else if (r0 / (1.0 - c) <= tol) {
      skip_series = true;
    } else {
      q0 = stat_at(ws, 1, 0, 2);
      b0_l1 = r0;
      // series on b' = r0, added to acc = D^{-1} x0
      CPAA_HIP(init_w1(pl, ws, ws.r, 1.0, true, false, true, st));
    }
  }
  if (!warm) {
    CPAA_HIP(fill_f64(ws.stat_slots, 0.0, (size_t)kSlots * ws.cols * kStat, st));
    CPAA_HIP(init_w1(pl, ws, dp, 1.0 - c, false, true, true, st));
    if ((s = read_back(ws, st)) != CPAA_OK) return s;
    if (!p_checked && (s = check_p_stats(ws, 0)) != CPAA_OK) return s;
    q0 = stat_at(ws, 0, 0, 2);
    b0_l1 = (1.0 - c) * stat_at(ws, 0, 0, 0);
    if (pl->opts.autotune && !pl->tuned_w1 && pl->maps.size() > 1 && !pl->sliced && !ext) {
      // autotune the work-item size on this input: time a few terms per candidate
      size_t best = 0;
      float best_ms = 1e30f;
      for (size_t i = 0; i < pl->maps.size(); ++i) {
        select_map(pl, i);
        hipError_t e = hipSuccess;
        time_terms(pl, ws, term_w1, 2, st, &e);            // warm-up
        const float ms = time_terms(pl, ws, term_w1, 4, st, &e);
        CPAA_HIP(e);
        if (ms < best_ms) {
          best_ms = ms;
          best = i;
        }
      }
      select_map(pl, best);
      pl->tuned_w1 = true;
      // restart the series (the probes overwrote z and acc)
      CPAA_HIP(init_w1(pl, ws, dp, 1.0 - c, false, true, true, st));
    }
    if (pl->opts.autotune && pl->opts.slice_shape == 0 && !pl->tuned_hub && pl->sliced &&
        pl->hub.built && !ext) {
      // launch shape of the hub-sliced gather pass: time a few terms with each
      // (the shape does not change a term's result)
      int best = pl->hub.cfg;
      float best_ms = 1e30f;
      for (int k = 0; k < kHubConfigs; ++k) {
        pl->hub.cfg = k;
        hipError_t e = hipSuccess;
        time_terms(pl, ws, term_w1, 2, st, &e);            // warm-up
        const float ms = time_terms(pl, ws, term_w1, 4, st, &e);
        CPAA_HIP(e);
        if (ms < best_ms) {
          best_ms = ms;
          best = k;
        }
      }
      pl->hub.cfg = best;
      pl->tuned_hub = true;
      CPAA_HIP(init_w1(pl, ws, dp, 1.0 - c, false, true, true, st));
    }
  }

  const double target_main = 0.5 * tol;
  int k_cap = 0;
  if (!skip_series) {
    k_cap = series_cap(pl, ws, q0, b0_l1, target_main);
    const int k_min = std::min(series_first_check(pl, ws, target_main, !warm), k_cap);
    if ((s = run_series(pl, ws, term_w1, 0, k_cap, k_min, target_main, timer, st)) != CPAA_OK)
      return s;
  }
  series_terms.push_back(k_cap);

  double bound = 0.0;
  // without normalize the last residual pass can write the result itself
  bool x_written = false;
  for (;;) {
    CPAA_HIP(fill_f64(ws.stat_slots + (size_t)kSlots * ws.cols * kStat, 0.0,
                      (size_t)kSlots * ws.cols * kStat, st));
    CPAA_HIP(residual_w1(pl, ws, st, pl->opts.normalize ? nullptr : dx, &x_written));
    if ((s = read_back(ws, st)) != CPAA_OK) return s;
    HostView hv = host_view(ws);
    const int ran = hv.done[0] ? hv.terms[0] : series_terms.back();
    series_terms.back() = skip_series && series_terms.size() == 1 ? 0 : ran;
    if (series_terms.size() == 1) {
      R.terms = series_terms[0];
    } else {
      R.refine_terms += series_terms.back();
    }
    R.series_cert = hv.series_cert[0];
    R.resid_l1 = stat_at(ws, 1, 0, 0);
    R.resid_max = stat_at(ws, 1, 0, 1);
    // the dropped vertices of a drop_isolated plan hold (1-c) p_v each
    R.mass = stat_at(ws, 1, 0, 3) + (1.0 - c) * stat_at(ws, 0, 0, 3);
    bound = rigorous_bound(pl, R.resid_l1, stat_at(ws, 1, 0, 4), R.mass);
    if (bound <= tol || !std::isfinite(bound) || R.refinements >= pl->opts.max_refine) break;
    // correction series on b' = r: x += x_M(r)
    const double target_ref = 0.25 * tol;
    const int kr = series_cap(pl, ws, stat_at(ws, 1, 0, 2), stat_at(ws, 1, 0, 0), target_ref);
    CPAA_HIP(init_w1(pl, ws, ws.r, 1.0, true, false, true, st));
    R.refinements++;
    series_terms.push_back(kr);
    if ((s = run_series(pl, ws, term_w1, (int)series_terms.size() - 1, kr,
                        std::min(series_first_check(pl, ws, target_ref, false), kr), target_ref,
                        timer, st)) != CPAA_OK)
      return s;
  }
  R.cert_bound = bound;
  R.certified = (bound <= tol) ? 1 : 0;
  const double scale = pl->opts.normalize ? 1.0 / R.mass : 1.0;
  if (!x_written) CPAA_HIP(finalize_w1(pl, ws, dx, scale, st));
  CPAA_HIP(dropped_out(pl, dp, (1.0 - c) * scale, dx, st));
  CPAA_HIP(hipEventRecord(pl->ev_end, st));
  if (!pl->opts.io_device)
    CPAA_HIP(hipMemcpyAsync(x, dx, n_io * sizeof(double), hipMemcpyDeviceToHost, st));
  CPAA_HIP(hipStreamSynchronize(st));
  float ms = 0.f;
  CPAA_HIP(hipEventElapsedTime(&ms, pl->ev_begin, pl->ev_end));
  R.ms_total = ms;
  timer.total(series_terms, &R.ms_terms, &R.term_launches);
  if (pl->opts.normalize) R.mass = 1.0;
  R.edges = pl->nnz * static_cast<int64_t>(R.terms + R.refine_terms);
  if (rep) *rep = R;
  if (!R.certified) {
    set_error("tolerance not certified: bound " + std::to_string(bound));
    return CPAA_ENOCONV;
  }
  return CPAA_OK;
}

// ----------------------------------------------------------------------------
// Batched solves: tiles of W right-hand sides, one SpMM kernel per term.
// ----------------------------------------------------------------------------
cpaa_status solve_batched(cpaa_plan_t pl, int32_t B, const double* P, int64_t ldp, double tol,
                          const double* X0, int64_t ldx0, double* X, int64_t ldx,
                          cpaa_report* reps, void* stream, Method method) {
  set_error("");
  if (pl && pl->directed) {
    if (!P || !X || B <= 0) {
      set_error("cpaa_solve_batched: null argument or B <= 0");
      return CPAA_EINVAL;
    }
    if (X0) {
      set_error("a directed plan has no warm start (X0 must be NULL)");
      return CPAA_EINVAL;
    }
    if (ldp < pl->n || ldx < pl->n) {
      set_error("leading dimensions must be >= n");
      return CPAA_EINVAL;
    }
    return solve_directed_columns(pl, B, P, ldp, tol, X, ldx, reps, stream);
  }
  if (!pl || !P || !X || B <= 0) {
    set_error("cpaa_solve_batched: null argument or B <= 0");
    return CPAA_EINVAL;
  }
  if (!(tol > 0.0) || !std::isfinite(tol)) {
    set_error("tol must be positive and finite");
    return CPAA_EINVAL;
  }
  if (pl->num_graphs > 1) {
    // a block-diagonal plan: one right-hand side per graph, stacked in one
    // vector (graph g's entries at its own vertices); reps gets one report per graph
    if (B != 1 || X0 != nullptr || method != Method::kChebyshev) {
      set_error("a block-diagonal plan takes B = 1 (one column holding every graph's "
                "personalization), no X0, CPAA only");
      return CPAA_EINVAL;
    }
    return cpaa_solve_graphs(pl, P, tol, X, reps, stream);
  }
  const int64_t n = pl->n;
  const int64_t n_io = pl->n_caller;
  if (ldp < n_io || ldx < n_io || (X0 && ldx0 < n_io)) {
    set_error("leading dimensions must be >= n");
    return CPAA_EINVAL;
  }
  if (pl->fp64 || pl->deterministic || pl->n_drop > 0)
    return solve_columns(pl, B, P, ldp, tol, X0, ldx0, X, ldx, reps, stream, method);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  cpaa_status s;
  if (pl->opts.autotune && pl->opts.tile_w == 0 && !pl->tuned_tile && pl->opts.io_device) {
    // autotune the tile width on this input: time a few terms per candidate
    int best_w = pl->tile_w;
    float best_ms = 1e30f;
    for (int Wc : {16, 32, 64}) {
      if (Wc > 16 && Wc / 2 >= B) break;
      const int Tc = (B + Wc - 1) / Wc;
      if ((s = ensure_workspace(pl, pl->wst, Wc, Tc)) != CPAA_OK) return s;
      pl->wst.method = method;
      CPAA_HIP(fill_f64(pl->wst.stat_slots, 0.0, (size_t)2 * kSlots * pl->wst.cols * kStat, st));
      CPAA_HIP(init_tile(pl, pl->wst, P, ldp, B, 1.0 - pl->c, false, false, true, st));
      hipError_t e = hipSuccess;
      time_terms(pl, pl->wst, term_tile, 2, st, &e);
      const float ms = time_terms(pl, pl->wst, term_tile, 4, st, &e) / (float)(Tc * Wc);
      CPAA_HIP(e);
      if (ms < best_ms) {
        best_ms = ms;
        best_w = Wc;
      }
    }
    pl->tile_w = best_w;
    pl->tuned_tile = true;
  }
  int W = pl->tile_w;
  while (W > 8 && W / 2 >= B) W /= 2;
  const int T = (B + W - 1) / W;
  s = ensure_workspace(pl, pl->wst, W, T);
  if (s != CPAA_OK) return s;
  Workspace& ws = pl->wst;
  ws.method = method;
  const double c = pl->c;
  const int64_t cols = ws.cols;

  TempDev tP, tX0, tX;
  const double* dP = P;
  const double* dX0 = X0;
  double* dX = X;
  int64_t lp = ldp, lx0 = ldx0, lx = ldx;
  if (!pl->opts.io_device) {
    const size_t bytes = (size_t)B * n * sizeof(double);
    if (hipMalloc(&tP.p, bytes) != hipSuccess || hipMalloc(&tX.p, bytes) != hipSuccess ||
        (X0 && hipMalloc(&tX0.p, bytes) != hipSuccess)) {
      (void)hipGetLastError();
      set_error("device allocation for host I/O failed");
      return CPAA_ENOMEM;
    }
    CPAA_HIP(hipMemcpy2DAsync(tP.p, n * sizeof(double), P, ldp * sizeof(double),
                              n * sizeof(double), B, hipMemcpyHostToDevice, st));
    if (X0)
      CPAA_HIP(hipMemcpy2DAsync(tX0.p, n * sizeof(double), X0, ldx0 * sizeof(double),
                                n * sizeof(double), B, hipMemcpyHostToDevice, st));
    dP = static_cast<const double*>(tP.p);
    dX0 = X0 ? static_cast<const double*>(tX0.p) : nullptr;
    dX = static_cast<double*>(tX.p);
    lp = lx0 = lx = n;
  }

  TermTimer timer{pl, pl->opts.time_kernels};
  std::vector<int> series_terms;
  std::vector<int> terms_main(T, 0), refine_terms(T, 0), refinements(T, 0);
  std::vector<int> fallback(cols, 0);
  std::vector<double> bound(cols, 0.0), r_l1(cols, 0.0), r_max(cols, 0.0), mass(cols, 0.0),
      q_r(cols, 0.0), scert(cols, -1.0);
  HostView hv = host_view(ws);

  CPAA_HIP(hipEventRecord(pl->ev_begin, st));
  CPAA_HIP(fill_f64(ws.stat_slots, 0.0, (size_t)2 * kSlots * cols * kStat, st));
  auto validate_cols = [&]() -> cpaa_status {
    for (int j = 0; j < B; ++j) {
      cpaa_status e = check_p_stats(ws, j);
      if (e != CPAA_OK) {
        set_error(std::string("column ") + std::to_string(j) + ": " + cpaa_last_error());
        return e;
      }
    }
    return CPAA_OK;
  };

  const double target_main = 0.5 * tol;
  int k_min;
  std::vector<double> q(cols, 0.0), b_l1(cols, 0.0);
  if (dX0) {
    CPAA_HIP(load_x0_tile(pl, ws, dX0, lx0, B, st));
    CPAA_HIP(init_tile(pl, ws, dP, lp, B, 1.0 - c, false, true, false, st));
    CPAA_HIP(residual_tile(pl, ws, nullptr, st));
    if ((s = read_back(ws, st)) != CPAA_OK) return s;
    if ((s = validate_cols()) != CPAA_OK) return s;
    for (int64_t j = 0; j < cols; ++j) {
      const double r0 = stat_at(ws, 1, j, 0);
      const double bnorm = (1.0 - c) * stat_at(ws, 0, j, 0);
      const bool finite = stat_at(ws, 0, j, 1) == 0.0 && stat_at(ws, 1, j, 5) == 0.0 &&
                          std::isfinite(r0);
      const bool use_warm = j < B && finite && r0 < bnorm;
      hv.plain[j] = use_warm ? 0 : 1;
      fallback[j] = (j < B && !use_warm) ? 1 : 0;
      q[j] = use_warm ? stat_at(ws, 1, j, 2) : stat_at(ws, 0, j, 2);
      b_l1[j] = use_warm ? r0 : bnorm;
    }
    CPAA_HIP(hipMemcpyAsync(ws.plain, hv.plain, cols * sizeof(int), hipMemcpyHostToDevice, st));
    CPAA_HIP(init_tile_from_r(pl, ws, nullptr, ws.plain, st));
    k_min = series_first_check(pl, ws, target_main, false);
  } else {
    CPAA_HIP(init_tile(pl, ws, dP, lp, B, 1.0 - c, false, true, true, st));
    if ((s = read_back(ws, st)) != CPAA_OK) return s;
    if ((s = validate_cols()) != CPAA_OK) return s;
    for (int64_t j = 0; j < cols; ++j) {
      q[j] = stat_at(ws, 0, j, 2);
      b_l1[j] = (1.0 - c) * stat_at(ws, 0, j, 0);
    }
    k_min = series_first_check(pl, ws, target_main, true);
  }
  int k_cap = 0;
  for (int64_t j = 0; j < cols; ++j)
    k_cap = std::max(k_cap, series_cap(pl, ws, q[j], b_l1[j], target_main));
  k_min = std::min(k_min, k_cap);
  if ((s = run_series(pl, ws, term_tile, 0, k_cap, k_min, target_main, timer, st)) != CPAA_OK)
    return s;
  series_terms.push_back(k_cap);

  std::vector<int> active(T, 1);
  bool first = true;
  bool masked = false;
  for (int round = 0;; ++round) {
    CPAA_HIP(fill_f64(ws.stat_slots + (size_t)kSlots * cols * kStat, 0.0,
                      (size_t)kSlots * cols * kStat, st));
    CPAA_HIP(residual_tile(pl, ws, masked ? ws.active : nullptr, st));
    if ((s = read_back(ws, st)) != CPAA_OK) return s;
    int ran_max = 0;
    for (int t = 0; t < T; ++t) {
      if (!active[t]) continue;
      const int ran = hv.terms[t];
      ran_max = std::max(ran_max, ran);
      if (first) terms_main[t] = ran;
      else refine_terms[t] += ran;
      for (int jj = 0; jj < W; ++jj) {
        const int64_t j = (int64_t)t * W + jj;
        r_l1[j] = stat_at(ws, 1, j, 0);
        r_max[j] = stat_at(ws, 1, j, 1);
        q_r[j] = stat_at(ws, 1, j, 2);
        mass[j] = stat_at(ws, 1, j, 3);
        scert[j] = hv.series_cert[j];
        bound[j] = rigorous_bound(pl, r_l1[j], stat_at(ws, 1, j, 4), mass[j]);
      }
    }
    series_terms.back() = ran_max;
    first = false;
    bool any = false;
    int k_ref = 0;
    const double target_ref = 0.25 * tol;
    for (int t = 0; t < T; ++t) {
      bool need = false;
      for (int jj = 0; jj < W; ++jj) {
        const int64_t j = (int64_t)t * W + jj;
        if (j < B && (bound[j] > tol) && std::isfinite(bound[j])) need = true;
      }
      active[t] = (need && refinements[t] < pl->opts.max_refine) ? 1 : 0;
      if (active[t]) {
        any = true;
        for (int jj = 0; jj < W; ++jj) {
          const int64_t j = (int64_t)t * W + jj;
          k_ref = std::max(k_ref, series_cap(pl, ws, q_r[j], r_l1[j], target_ref));
        }
      }
    }
    if (!any) break;
    for (int t = 0; t < T; ++t) {
      hv.active[t] = active[t];
      refinements[t] += active[t];
    }
    CPAA_HIP(hipMemcpyAsync(ws.active, hv.active, T * sizeof(int), hipMemcpyHostToDevice, st));
    masked = true;
    CPAA_HIP(init_tile_from_r(pl, ws, ws.active, nullptr, st));
    series_terms.push_back(k_ref);
    if ((s = run_series(pl, ws, term_tile, (int)series_terms.size() - 1, k_ref,
                        std::min(series_first_check(pl, ws, target_ref, false), k_ref),
                        target_ref, timer, st, ws.active)) != CPAA_OK)
      return s;
  }
  const double* col_scale = nullptr;
  if (pl->opts.normalize) {
    for (int64_t j = 0; j < cols; ++j) hv.col_scale[j] = mass[j] != 0.0 ? 1.0 / mass[j] : 1.0;
    CPAA_HIP(hipMemcpyAsync(ws.col_scale, hv.col_scale, cols * sizeof(double),
                            hipMemcpyHostToDevice, st));
    col_scale = ws.col_scale;
  }
  CPAA_HIP(finalize_tile(pl, ws, dX, lx, B, col_scale, st));
  CPAA_HIP(hipEventRecord(pl->ev_end, st));
  if (!pl->opts.io_device)
    CPAA_HIP(hipMemcpy2DAsync(X, ldx * sizeof(double), dX, n * sizeof(double), n * sizeof(double),
                              B, hipMemcpyDeviceToHost, st));
  CPAA_HIP(hipStreamSynchronize(st));
  float ms = 0.f;
  CPAA_HIP(hipEventElapsedTime(&ms, pl->ev_begin, pl->ev_end));
  double ms_terms = 0.0;
  int64_t launches = 0;
  timer.total(series_terms, &ms_terms, &launches);
  bool all_ok = true;
  for (int j = 0; j < B; ++j) {
    const int t = j / W;
    cpaa_report R;
    std::memset(&R, 0, sizeof(R));
    R.method = method == Method::kPower ? 1 : 0;
    R.terms = terms_main[t];
    R.refine_terms = refine_terms[t];
    R.refinements = refinements[t];
    R.cert_bound = bound[j];
    R.certified = bound[j] <= tol ? 1 : 0;
    R.fallback_used = fallback[j];
    R.resid_l1 = r_l1[j];
    R.resid_max = r_max[j];
    R.mass = pl->opts.normalize ? 1.0 : mass[j];
    R.series_cert = scert[j];
    R.ms_total = ms;
    R.ms_terms = ms_terms;
    R.term_launches = launches;
    R.edges = pl->nnz * static_cast<int64_t>(R.terms + R.refine_terms);
    all_ok = all_ok && R.certified;
    if (reps) reps[j] = R;
  }
  if (!all_ok) {
    set_error("tolerance not certified for every column");
    return CPAA_ENOCONV;
  }
  return CPAA_OK;
}

// The power method on a directed plan (kernels_w1.hip, x-space): the series
// runs from x_0 = p; a correction runs the same iteration on b = r from
// x_0 = r/(1-c); certification as for the other solves (FP64 residual of P'').
cpaa_status solve_directed(cpaa_plan_t pl, const double* p, double tol, double* x,
                           cpaa_report* rep, void* stream) {
  if (!p || !x) {
    set_error("cpaa_solve_power: null argument");
    return CPAA_EINVAL;
  }
  if (!(tol > 0.0) || !std::isfinite(tol)) {
    set_error("tol must be positive and finite");
    return CPAA_EINVAL;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  cpaa_status s = ensure_workspace(pl, pl->ws1, 1, 1);
  if (s != CPAA_OK) return s;
  Workspace& ws = pl->ws1;
  ws.method = Method::kPower;
  const int n = pl->n;
  const double c = pl->c;
  TempDev tp, tx;
  const double* dp = p;
  double* dx = x;
  if (!pl->opts.io_device) {
    if (hipMalloc(&tp.p, n * sizeof(double)) != hipSuccess ||
        hipMalloc(&tx.p, n * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      set_error("device allocation for host I/O failed");
      return CPAA_ENOMEM;
    }
    CPAA_HIP(hipMemcpyAsync(tp.p, p, n * sizeof(double), hipMemcpyHostToDevice, st));
    dp = static_cast<const double*>(tp.p);
    dx = static_cast<double*>(tx.p);
  }
  TermTimer timer{pl, pl->opts.time_kernels};
  std::vector<int> series_terms;
  cpaa_report R;
  std::memset(&R, 0, sizeof(R));
  R.method = 1;
  CPAA_HIP(hipEventRecord(pl->ev_begin, st));
  CPAA_HIP(fill_f64(ws.stat_slots, 0.0, (size_t)2 * kSlots * ws.cols * kStat, st));
  CPAA_HIP(fill_f64(ws.dang, 0.0, 3 * kSlots, st));
  CPAA_HIP(init_dir(pl, ws, dp, 1.0, false, true, st));
  if ((s = read_back(ws, st)) != CPAA_OK) return s;
  if ((s = check_p_stats(ws, 0)) != CPAA_OK) return s;
  const double target_main = 0.5 * tol;
  ws.dir_x0 = ws.b;    // x_0 = p = b/(1-c), in the plan's labels
  ws.dir_x0_scale = 1.0 / (1.0 - c);
  int k_cap = series_cap(pl, ws, 0.0, (1.0 - c) * stat_at(ws, 0, 0, 0), target_main);
  if ((s = run_series(pl, ws, term_dir, 0, k_cap, 0, target_main, timer, st)) != CPAA_OK) return s;
  series_terms.push_back(k_cap);
  double bound = 0.0;
  for (;;) {
    CPAA_HIP(fill_f64(ws.stat_slots + (size_t)kSlots * ws.cols * kStat, 0.0,
                      (size_t)kSlots * ws.cols * kStat, st));
    CPAA_HIP(residual_dir(pl, ws, st));
    if ((s = read_back(ws, st)) != CPAA_OK) return s;
    HostView hv = host_view(ws);
    const int ran = hv.done[0] ? hv.terms[0] : series_terms.back();
    series_terms.back() = ran;
    if (series_terms.size() == 1) R.terms = ran;
    else R.refine_terms += ran;
    R.series_cert = hv.series_cert[0];
    R.resid_l1 = stat_at(ws, 1, 0, 0);
    R.resid_max = stat_at(ws, 1, 0, 1);
    // the dropped vertices of a drop_isolated plan hold (1-c) p_v each
    R.mass = stat_at(ws, 1, 0, 3) + (1.0 - c) * stat_at(ws, 0, 0, 3);
    bound = rigorous_bound(pl, R.resid_l1, stat_at(ws, 1, 0, 4), R.mass);
    if (bound <= tol || !std::isfinite(bound) || R.refinements >= pl->opts.max_refine) break;
    // correction: the same iteration on b' = r from x_0 = r/(1-c), added to acc
    const double target_ref = 0.25 * tol;
    const int kr = series_cap(pl, ws, 0.0, R.resid_l1, target_ref);
    CPAA_HIP(fill_f64(ws.dang, 0.0, 3 * kSlots, st));
    CPAA_HIP(init_dir(pl, ws, ws.r, 1.0 / (1.0 - c), true, false, st));
    ws.dir_x0 = ws.r;
    ws.dir_x0_scale = 1.0 / (1.0 - c);
    R.refinements++;
    series_terms.push_back(kr);
    if ((s = run_series(pl, ws, term_dir, (int)series_terms.size() - 1, kr, 0, target_ref, timer,
                        st)) != CPAA_OK)
      return s;
  }
  R.cert_bound = bound;
  R.certified = (bound <= tol) ? 1 : 0;
  const double scale = pl->opts.normalize ? 1.0 / R.mass : 1.0;
  CPAA_HIP(finalize_dir(pl, ws, dx, scale, st));
  CPAA_HIP(hipEventRecord(pl->ev_end, st));
  if (!pl->opts.io_device)
    CPAA_HIP(hipMemcpyAsync(x, dx, n * sizeof(double), hipMemcpyDeviceToHost, st));
  CPAA_HIP(hipStreamSynchronize(st));
  float ms = 0.f;
  CPAA_HIP(hipEventElapsedTime(&ms, pl->ev_begin, pl->ev_end));
  R.ms_total = ms;
  timer.total(series_terms, &R.ms_terms, &R.term_launches);
  if (pl->opts.normalize) R.mass = 1.0;
  R.edges = pl->nnz * static_cast<int64_t>(R.terms + R.refine_terms);
  if (rep) *rep = R;
  if (!R.certified) {
    set_error("tolerance not certified: bound " + std::to_string(bound));
    return CPAA_ENOCONV;
  }
  return CPAA_OK;
}

// ---- the no-allocation entry point ----
// A fixed device array backs the single-vector workspace of cpaa_solve_noalloc.
// In host code `scratch` names a host-side stand-in, never the device array:
// its device address (one per device) comes from hipGetSymbolAddress, taken
// once per device with that device current, and only that address is used.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};
// host mirrors of the statistics and stop flags (pageable; calls that overlap race)
alignas(256) unsigned char g_noalloc_host[1024];
alignas(64) int g_noalloc_poll[2];

cpaa_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxScratchDevices) {
    set_error("cpaa_solve_noalloc: device index out of range");
    return CPAA_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      set_error(std::string("cpaa_solve_noalloc: hipGetSymbolAddress(scratch) failed: ") +
                hipGetErrorString(e));
      return CPAA_EDEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return CPAA_OK;
}

cpaa_status solve_noalloc(cpaa_plan_t pl, const double* p, double tol, const double* x0,
                          double* x, cpaa_report* rep, void* stream) {
  set_error("");
  if (!pl || !p || !x) {
    set_error("cpaa_solve_noalloc: null argument");
    return CPAA_EINVAL;
  }
  if (pl->directed || pl->num_graphs > 1) {
    set_error("cpaa_solve_noalloc: undirected single-graph plans only");
    return CPAA_EINVAL;
  }
  if (!pl->opts.io_device) {
    set_error("cpaa_solve_noalloc: p, x0 and x must be device pointers (io_device = 1)");
    return CPAA_EINVAL;
  }
  int dev = -1;
  CPAA_HIP(hipGetDevice(&dev));
  if (dev != pl->device) {
    set_error("cpaa_solve_noalloc: the plan's device must be current");
    return CPAA_EINVAL;
  }
  // the workspace's size first (a counting layout), then the same layout in the
  // array; the FP64 partials of the hub-sliced residual are included when they
  // fit (the residual of the allocating entry point, so deterministic plans
  // return the same bits from both), else the residual runs in row order
  auto count = [&](bool resid64) {
    size_t need = 0;
    Workspace probe;
    layout_workspace(
        pl, probe, 1, 1,
        [&](void** ptr, size_t bytes) {
          need = (need + 255) & ~size_t(255);
          need += bytes ? bytes : 8;
          *ptr = nullptr;
          return true;
        },
        resid64);
    return need;
  };
  bool resid64 = true;
  size_t need = count(true);
  if (need > kScratchBytes) {
    resid64 = false;
    need = count(false);
  }
  if (need > kScratchBytes) {
    set_error("cpaa_solve_noalloc: this plan needs " + std::to_string(need) +
              " bytes of workspace, the static array holds " + std::to_string(kScratchBytes) +
              " (n = " + std::to_string(pl->n) + ")");
    return CPAA_EINVAL;
  }
  if (host_mirror_bytes(1, 1) > sizeof(g_noalloc_host)) {
    set_error("cpaa_solve_noalloc: host mirror too small");
    return CPAA_EINVAL;
  }
  void* base = nullptr;
  cpaa_status s = scratch_address(dev, &base);
  if (s != CPAA_OK) return s;
  Workspace ws;
  size_t off = 0;
  layout_workspace(
      pl, ws, 1, 1,
      [&](void** ptr, size_t bytes) {
        off = (off + 255) & ~size_t(255);
        *ptr = static_cast<unsigned char*>(base) + off;
        off += bytes ? bytes : 8;
        return true;
      },
      resid64);
  ws.external = true;
  ws.host = reinterpret_cast<double*>(g_noalloc_host);
  ws.host_bytes = host_mirror_bytes(1, 1);
  ws.poll_host = g_noalloc_poll;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // the array keeps the last call's contents: clear what must start at zero
  if ((s = zero_workspace(ws, pl, true, st)) != CPAA_OK) return s;
  return solve_single(pl, p, tol, x0, x, rep, stream, Method::kChebyshev, &ws);
}

}  // namespace

extern "C" cpaa_status cpaa_solve_noalloc(cpaa_plan_t pl, const double* p, double tol,
                                          const double* x0, double* x, cpaa_report* rep,
                                          void* stream) {
  return solve_noalloc(pl, p, tol, x0, x, rep, stream);
}

extern "C" cpaa_status cpaa_solve(cpaa_plan_t pl, const double* p, double tol, const double* x0,
                                  double* x, cpaa_report* rep, void* stream) {
  return solve_single(pl, p, tol, x0, x, rep, stream, Method::kChebyshev);
}

extern "C" cpaa_status cpaa_solve_power(cpaa_plan_t pl, const double* p, double tol,
                                        const double* x0, double* x, cpaa_report* rep,
                                        void* stream) {
  return solve_single(pl, p, tol, x0, x, rep, stream, Method::kPower);
}

extern "C" cpaa_status cpaa_solve_batched(cpaa_plan_t pl, int32_t B, const double* P, int64_t ldp,
                                          double tol, const double* X0, int64_t ldx0, double* X,
                                          int64_t ldx, cpaa_report* reps, void* stream) {
  return solve_batched(pl, B, P, ldp, tol, X0, ldx0, X, ldx, reps, stream, Method::kChebyshev);
}

extern "C" cpaa_status cpaa_solve_power_batched(cpaa_plan_t pl, int32_t B, const double* P,
                                                int64_t ldp, double tol, const double* X0,
                                                int64_t ldx0, double* X, int64_t ldx,
                                                cpaa_report* reps, void* stream) {
  return solve_batched(pl, B, P, ldp, tol, X0, ldx0, X, ldx, reps, stream, Method::kPower);
}
