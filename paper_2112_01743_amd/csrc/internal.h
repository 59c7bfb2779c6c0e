// Internal declarations of the CPAA library (gfx950 / HIP).
//
// Data layout in HBM (single-graph plan):
//   row_ptr[n+1], col_idx[nnz]      int32 CSR pattern (caller's vertex order)
//   z[3][n]                          FP32 Chebyshev vectors in z-space, z_k = D^{-1} T_k(P) b
//   acc[n]                           FP64 running sum D^{-1} x_M
//   b[n], r[n]                       FP64 right-hand side and residual
// Batched solves use tiles of W right-hand sides: z[3][tiles][n][W] (FP32),
// acc/b/r[tiles][n][W] (FP64), so the W values of one vertex are contiguous and
// a neighbour gather is one coalesced W*4-byte access.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "cpaa.h"

namespace cpaa {

constexpr int kWG = 256;           // threads per workgroup
constexpr int kSlots = 64;         // atomic reduction slots (spread contention)
constexpr int kMaxTerms = 512;     // hard cap on terms of one series
constexpr int kStat = 6;           // reduction fields per column (see kernels.hip)
constexpr int kLongRow = 128;      // W = 1: rows longer than this never share a block with short rows
constexpr int kTileLongDeg = 512;  // tiled: rows above this degree are split across wavefronts
constexpr int kTileChunkNnz = 256; // tiled: nnz per wavefront chunk of a split row
constexpr int kTileShortNnz = 128; // tiled: nnz budget of a wavefront's group of short rows
constexpr int kGraphClasses = 4;   // multi-graph: size classes (LDS per workgroup) launched in turn

void set_error(const std::string& msg);

#define CPAA_HIP(call)                                                            \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ::cpaa::set_error(std::string("HIP error: ") + hipGetErrorString(e_) +      \
                        " at " + __FILE__ + ":" + std::to_string(__LINE__));      \
      return CPAA_EDEVICE;                                                        \
    }                                                                             \
  } while (0)

// Work unit of the single-vector SpMV kernels: a window of at most
// kWG * npt stored entries.
//   row1 >= 0: rows [row0, row1), all of whose entries lie in [nnz0, nnz1).
//   row1 <  0: one chunk [nnz0, nnz1) of the split row row0; its partial sum
//              goes to slot -(row1 + 1).
struct WorkItem {
  int row0;
  int row1;
  int nnz0;
  int nnz1;
};

// Column-sliced single-vector term (one column slice per XCD).  Vertices are
// relabelled so that slice s is the contiguous label range
// [slice_off[s], slice_off[s+1]); slice s's stored entries (row order) are
// packed as (column - slice_off[s]) << row_bits | (row - item.row0), with
// row_bits = 12 when every slice has fewer than 2^20 - 1 vertices, else 11.
// Chunks of rows split across workgroups store the plain local column.
constexpr int kSlices = 8;           // XCDs of the chip
constexpr int kSliceRowBitsMax = 12;
constexpr int kSliceRowsMax = 1 << kSliceRowBitsMax;   // LDS row sums of a sliced work item
constexpr int kSliceNpt = 32;        // entries per thread of a sliced work item
// with 11 row bits local columns stay below 2^21 - 1, so no packed entry
// equals kSliceNone (slices hold at most n/8 + 8 vertices)
constexpr int64_t kSliceMaxN = int64_t(kSlices) * ((int64_t(1) << 21) - 16);
constexpr uint32_t kSliceNone = 0xFFFFFFFFu;   // padding entry
constexpr int kSliceHub = 2048;      // leading vertices of a slice cached in LDS per work item

struct SlicedMap {
  uint32_t* d_entries = nullptr;     // [nnz] slice-major
  WorkItem* d_items = nullptr;       // slice-major; nnz offsets index d_entries
  int item_off[kSlices + 1] = {};    // items of slice s: [item_off[s], item_off[s+1])
  int max_items = 0;                 // most items in one slice
  int slice_off[kSlices + 1] = {};   // vertex labels of slice s
  int row_bits = 11;                 // local row field of a packed entry
  int n_split_rows = 0;
  int* d_split_nchunks = nullptr;    // [n_split_rows]
};

// Hub-sliced single-vector term (undirected plans with column slices; the
// layout above stays in use for directed plans).  Per column slice s only the
// rows with at least one entry in s ("present" rows) get a partial sum, stored
// compactly: row u's partial for slice s sits at part[pofs[s] + j_s(u)], j_s(u)
// = number of present rows of s before u.  mask[u] holds one bit per slice,
// and base[b][s] = j_s of the first present row at or after row 64 b, so the
// combine pass finds every partial of a 64-row block from a ballot.  The
// gather pass runs workgroups of several wavefronts, each on one slice, that
// copy the slice's first `hub` vertices (its highest degrees) to LDS once for
// their wavefronts, each of which takes one wave item: at most
// kHubItemCap entries and kHubRows consecutive present rows, entries packed as
// local column << kHubRowBits | (j - j0), lane l owning the contiguous run
// [l RL, (l+1) RL) of the item's entries, stored transposed (element i of the
// run at i * 64 + l).  A row with more than kHubItemCap entries in a slice is
// cut into chunk items (plain local columns); the last chunk to finish adds
// the chunk sums in chunk order.
constexpr int kHubNpt = 32;                  // entries per lane of a wave item
// the gather kernel keeps a lane's row starts in one 32-bit mask, and the run
// layout loads four entries at a time
static_assert(kHubNpt <= 32 && kHubNpt % 4 == 0, "entries per lane of a wave item");
constexpr int kHubItemCap = 64 * kHubNpt;    // entries per wave item
constexpr int kHubRowBits = 11;              // packed row field (j - j0 < kHubRows)
constexpr int kHubRows = 1024;               // present rows per wave item (LDS row sums)
// LDS row sums are padded by one word per 32 (row r at r + r / 32): the rows a
// lane finishes step by its run length, which would otherwise put the lanes
// of a store on a few banks
constexpr int kHubRowsPad = kHubRows + kHubRows / 32;
constexpr int kHubConfigs = 4;               // launch shapes (waves per workgroup, hub size)
#ifdef CPAA_TEST_SLICE_ENTRY_LIMIT
constexpr int64_t kSliceEntryLimit = CPAA_TEST_SLICE_ENTRY_LIMIT;   // test builds only
#else
constexpr int64_t kSliceEntryLimit = INT32_MAX;   // int32 entry offsets of the work items
#endif

// Launch shapes of the hub-sliced gather pass: wavefronts per workgroup and
// hub vertices in LDS (one copy per workgroup, shared by its wavefronts).  LDS
// per workgroup: waves * kHubRowsPad * 4 + hub * 4 bytes (gfx950: at most
// 160 KB).  Measured on the 4M-vertex power-law graph (gather pass per term):
// 16 / 22,528 175 us, 16 / 16,384 185 us, 8 / 8,192 189 us, 4 / 2,048 228 us;
// 12 wavefronts with a larger hub (24,576 or 27,648) 187 us: below 16
// wavefronts per CU the gathers in flight drop more than the hub gains; two
// workgroups per CU of 12 / 7,808 tie the best (175 us, 24 wavefronts per CU,
// half the hub), 10 / 9,920 183 us, and 512-row items with 12 / 14,144 179 us.
// A persistent variant (workgroups looping over items claimed from a counter)
// took 420-540 us; one with a workgroup per CU taking a fixed contiguous share
// of its slice's items (no counter, the hub copied once) about 187 us (the
// term 218 against 206 us); the per-item layout's pass 219 us.
struct HubShape {
  int waves, hub;   // one workgroup per `waves` consecutive wave items of a slice
};
constexpr HubShape kHubShapes[kHubConfigs] = {{16, 16384}, {8, 8192}, {4, 2048}, {16, 22528}};
// slice_shape 1-kHubConfigs selects a shape above, kHubConfigs + 1 the per-item
// layout (SlicedMap); 0 takes kSliceShapeAuto, or with autotune the fastest of
// the shapes above on the first solve.  Every shape sums a row's entries in the
// same order (the order is fixed by the map, not by the launch), so the shape
// changes the time of a term, never its result.
constexpr int kSliceShapeAuto = 1;
// The FP64 residual's gather pass on the same map: doubles in LDS, so a
// smaller hub per workgroup.  Measured on the 4M-vertex power-law graph:
// 12 / 7,168 253 us, 12 / 4,096 258 us, 16 / 2,048 299-309 us (its registers
// spill at 16 wavefronts), 8 / 4,096 305 us, 16 / 1,024 310 us, 8 / 8,192
// 320 us, 4 / 14,336 622 us.
constexpr HubShape kHubResidShape = {12, 7168};
inline int hub_groups_per_slice(int k, int max_items) {
  return (max_items + kHubShapes[k].waves - 1) / kHubShapes[k].waves;
}

// Run layout of a wave item: L entries, lane l owning the logical run
// [l RL, (l+1) RL), RL a multiple of 4, and element i of lane l's run stored at
// hub_slot(l, i), so that each lane reads 4 consecutive run elements with one
// 16-byte load and a wavefront's load covers 1 KB contiguously.
__host__ __device__ inline int hub_run_length(int L) { return ((L + 255) >> 8) << 2; }
__host__ __device__ inline int hub_slot(int lane, int i) {
  return (i >> 2) * 256 + lane * 4 + (i & 3);
}

struct HubItem {
  int j0;     // first present row of the item (slice-local compact index)
  int e0;     // first packed entry (global index into the entry array)
  int len;    // entries of the item (the run layout pads to a multiple of 64)
  int rows;   // present rows j0 .. j0 + rows - 1; < 0: chunk -(rows + 1) of a long row
};

struct HubMap {
  uint32_t* d_entries = nullptr;
  HubItem* d_items = nullptr;
  int item_off[kSlices + 1] = {};      // items of slice s
  int pofs[kSlices + 1] = {};          // partial sums of slice s: part[pofs[s] .. pofs[s+1])
  uint8_t* d_mask = nullptr;           // [n] bit s: row present in slice s
  int* d_base = nullptr;               // [ceil(n / 64)][kSlices]
  int groups[kHubConfigs] = {};        // workgroups per slice of each launch shape
  int groups_resid = 0;                // workgroups per slice of kHubResidShape
  // [n] sum over the neighbours u of v of (d_u + 3): the weight of |acc_v| in the
  // residual's rounding bound, which the hub-sliced residual adds per vertex
  double* d_wround = nullptr;
  int cfg = 0;                         // launch shape in use
  int n_long = 0;                      // rows cut into chunks
  int n_chunks = 0;
  int* d_chunk_long = nullptr;         // [n_chunks] long row of each chunk
  int* d_long_first = nullptr;         // [n_long] first chunk
  int* d_long_nch = nullptr;           // [n_long] chunks
  int* d_long_out = nullptr;           // [n_long] index of the row's partial in part
  bool built = false;
};

// One decomposition of the CSR into single-vector work items (for one npt).
struct WorkMap {
  int npt = 0;
  WorkItem* d_items = nullptr;
  int n_items = 0;
  int n_split_rows = 0;
  int* d_split_nchunks = nullptr;
};

// The series a solve sums on the term kernels (z_k in z-space, x = D acc).
//   kChebyshev (Alg. 1): z_1 = D^{-1}A z_0, z_{k+1} = 2 D^{-1}A z_k - z_{k-1};
//     acc = c_0/2 z_0 + sum c_k z_k; certificate partial d |z_{k+1} - beta z_k|.
//   kPower: the power method x_{t+1} = cPx_t + b started at x_0 = b/(1-c) (for
//     b = (1-c)p: eq. 2.1 iterated from p), summed as x_0 plus its increments
//     delta_t = x_{t+1} - x_t = (cP)^t delta_0, delta_0 = c(P - I)x_0.  With
//     z_0 = D^{-1}b: z_1 = c(D^{-1}A z_0 - z_0) = (1-c) D^{-1}delta_0 and
//     z_{k+1} = c D^{-1}A z_k; every coefficient is 1/(1-c), so acc after the
//     launch producing z_{k+1} is D^{-1}x_{k+1}.  Certificate partial
//     d |z_{k+1}| = (1-c) |delta_k|, and ||x_k - x*||_1 <= ||delta_k||_1/(1-c)
//     because delta_k is the residual b - (I-cP)x_k.
enum class Method { kChebyshev, kPower };

struct Workspace {
  Method method = Method::kChebyshev;  // series of the solve in progress
  int W = 0;              // tile width (1 = single vector path)
  int tiles = 0;
  int64_t cols = 0;       // tiles * W
  size_t vec_elems = 0;   // n * cols
  float* z[3] = {nullptr, nullptr, nullptr};
  double* acc = nullptr;
  double* b = nullptr;
  double* r = nullptr;
  double* slots = nullptr;       // [kMaxTerms+2][kSlots][cols] certificate partials
  double* stat_slots = nullptr;  // [kSlots][cols][kStat]
  double* stat = nullptr;        // [cols][kStat] collapsed
  int* done = nullptr;           // [tiles]
  int* terms = nullptr;          // [tiles]
  double* series_cert = nullptr; // [cols]
  float* part = nullptr;         // column-sliced term: [kSlices][n] FP32 partial row sums
                                 // (directed plans), or the compact partials of HubMap
  double* det_part = nullptr;    // deterministic plans: per-block partial sums (4 x blocks)
  int* det_count = nullptr;      // deterministic plans: arrival counter of those sums
  double* det_chunk = nullptr;   // deterministic plans: [split rows][det_max_chunks][2] chunk
                                 // sums of the residual's split rows
  int det_max_chunks = 0;
  double* det_defer = nullptr;   // deterministic plans: [split rows][3] (sum, sum of |.|, row)
  float* chunk_val = nullptr;    // hub-sliced term: [n_chunks] sums of long-row chunks
  double* part64 = nullptr;      // hub-sliced plans: compact FP64 partial sums of the residual
  double* chunk64 = nullptr;     // hub-sliced plans: [n_chunks] FP64 long-row chunk sums
  int* long_cnt = nullptr;       // hub-sliced term: [n_long] chunk arrivals
  double* dang = nullptr;        // directed plans: [5][kSlots] dangling mass of the increment
                                 // in z[0..2], then of x and |x| for the residual
  double* wdir = nullptr;        // directed plans: [n] FP64 D_out^+ x for the residual
  double* part_d = nullptr;      // column-sliced directed plans: [kSlices][n][2] FP64 partial
                                 // sums of w and |w| (residual)
  const double* dir_x0 = nullptr;  // directed power method: start of the series in progress
  double dir_x0_scale = 1.0;       //   x_0 = dir_x0_scale * dir_x0
  float* split_f = nullptr;      // [split slots * W] FP32 partial sums
  double* split_d = nullptr;     // [split slots * W] FP64 partial sums (residual)
  int* split_count = nullptr;    // [split slots] arrivals
  int* active = nullptr;         // [tiles] device copy of the tile mask of a correction pass
  int* plain = nullptr;          // [cols] columns restarted as plain solves
  double* col_scale = nullptr;   // [cols] output scale per column
  double* host = nullptr;        // pinned host mirror
  int* poll_host = nullptr;      // pinned [2][tiles] stop flags of a series read while it runs
  size_t host_bytes = 0;
  size_t split_elems = 0;        // split-row slots (all tiles)
  bool external = false;         // buffers owned by someone else (never freed here)
};

}  // namespace cpaa

struct cpaa_plan_s {
  int device = 0;
  int32_t n = 0;
  int64_t nnz = 0;
  double c = 0.85;
  double beta = 0.0;  // beta of the expansion in use (of c', below)
  double s = 0.0;     // sqrt(1-c'^2)
  double lam_lo = -1.0;  // expansion interval [lam_lo, 1]; c' = c(1-a)/(2A), A below
  double cheb_A = 1.0;   // 1 - c(1+a)/2
  double vol = 0.0;
  int max_deg = 0;
  int min_deg = 0;
  cpaa_opts opts{};
  int num_graphs = 1;

  int32_t* d_row_ptr = nullptr;
  int32_t* d_col_idx = nullptr;

  // single-vector path: its own labelling of the graph (relabelled when
  // column-sliced; otherwise these alias d_row_ptr / d_col_idx)
  int32_t* d_rp_w1 = nullptr;
  int32_t* d_ci_w1 = nullptr;
  int32_t* d_perm = nullptr;         // [n] single-vector label -> caller's label, or null
  int32_t n_caller = 0;              // the caller's vertex count (n plus dropped vertices)
  int32_t n_drop = 0;                // edgeless vertices dropped (opts.drop_isolated)
  int32_t* d_dropped = nullptr;      // [n_drop] their labels in the caller's numbering
  int reordered = 0;                 // 0 caller's labels, 1 column slices, 2 reverse Cuthill-McKee
  bool directed = false;             // rows list in-neighbours; solved by the power method only
  int32_t* d_dout = nullptr;         // directed plans: [n] out-degrees
  bool fp64 = false;                 // FP64 recurrence (opts.fp64_recurrence): row order only
  bool deterministic = false;        // opts.deterministic
  bool sliced = false;
  cpaa::SlicedMap slc;               // directed plans
  cpaa::HubMap hub;                  // undirected plans

  // single-vector work map in use (one of `maps`)
  int npt = 8;                       // nnz per thread of a work item
  cpaa::WorkItem* d_items = nullptr;
  int n_items = 0;
  int n_split_rows = 0;
  int* d_split_nchunks = nullptr;    // [n_split_rows]
  std::vector<cpaa::WorkMap> maps;   // candidates (several when autotuning)
  int max_split_rows = 0;            // over all candidates (workspace sizing)
  bool tuned_w1 = false;
  bool tuned_hub = false;            // launch shape of the hub-sliced gather pass chosen
  bool tuned_tile = false;
  int xcd_remap = 0;                 // single-vector kernels
  int xcd_remap_tile = 1;            // tiled kernels

  // tiled work map (per wavefront)
  cpaa::WorkItem* d_titems = nullptr;
  int n_titems = 0;
  int n_tsplit_rows = 0;
  int* d_tsplit_nchunks = nullptr;
  int tile_w = 64;

  // multi-graph batch
  int32_t* d_graph_ptr = nullptr;
  int32_t* d_graph_order = nullptr;  // graphs by size class, then by nnz, largest first
  int* d_queue = nullptr;            // [kGraphClasses] work counters
  int graph_cls_off[cpaa::kGraphClasses + 1] = {};   // graphs of class k: order[graph_cls_off[k] .. [k+1])
  int graph_cls_n[cpaa::kGraphClasses] = {};         // largest vertex count in class k (LDS sizing)
  int max_graph_n = 0;
  int64_t max_graph_nnz = 0;
  std::vector<int32_t> h_graph_ptr;
  std::vector<int64_t> h_graph_nnz;  // stored entries per graph
  void* graph_state = nullptr;       // graphs.hip: packed local pairs, records, HIP graph

  std::vector<double> ck;            // c_k, k = 0..kMaxTerms+1
  std::vector<double> pk;            // power-method coefficients 1/(1-c), k = 0..kMaxTerms+1

  cpaa::Workspace ws1;               // W = 1
  cpaa::Workspace wst;               // tiled
  cpaa::Workspace wsg;               // multi-graph

  hipEvent_t ev_begin = nullptr, ev_end = nullptr;
  hipEvent_t ev_poll[2] = {nullptr, nullptr};   // chunked power-method series
  std::vector<hipEvent_t> ev_terms;  // pairs around term launches
};

namespace cpaa {

// Weight of z_0 in acc and the coefficients of z_1, z_2, ... for the series
// of the solve in progress.
inline double series_a0(const cpaa_plan_s* pl, const Workspace& ws) {
  return ws.method == Method::kPower ? pl->pk[0] : pl->ck[0] / 2.0;
}
inline const std::vector<double>& series_coef(const cpaa_plan_s* pl, const Workspace& ws) {
  return ws.method == Method::kPower ? pl->pk : pl->ck;
}

// Epilogue constants of a term launch: z_{k+1} = alpha D^{-1}(A z_k) - gamma_c z_k
// - gamma zp, certificate partial d |z_{k+1} - beta z_k|; zp is z_{k-1}, or z_k
// itself for the power method's first launch.
struct TermShape {
  float alpha, gamma_c, gamma;  // z_{k+1} = alpha D^{-1}A z_k - gamma_c z_k - gamma zp
  double beta;
  bool zp_is_cur;
  double alpha_d, gamma_c_d, gamma_d;   // the same constants for the FP64 recurrence
};
inline TermShape term_shape(const cpaa_plan_s* pl, const Workspace& ws, bool first) {
  if (ws.method == Method::kPower) {
    const double c = pl->c;
    const float cf = static_cast<float>(c);
    return {cf, 0.f, first ? cf : 0.f, 0.0, first, c, 0.0, first ? c : 0.0};
  }
  // T_1 = t(P) T_0, T_{k+1} = 2 t(P) T_k - T_{k-1}, t(P) = (2P - (1+a)I)/(1-a)
  const double a = pl->lam_lo;
  const double al = 2.0 / (1.0 - a);
  const double gc = (1.0 + a) / (1.0 - a);
  const double A = first ? al : 2.0 * al, G = first ? gc : 2.0 * gc, P = first ? 0.0 : 1.0;
  return {static_cast<float>(A), static_cast<float>(G), static_cast<float>(P), pl->beta, false,
          A, G, P};
}

hipError_t fill_f64(double* p, double v, size_t count, hipStream_t st);
hipError_t fill_i32(int* p, int v, size_t count, hipStream_t st);
hipError_t collapse_stats(Workspace& ws, hipStream_t st);

// What one term launch (producing z_{k+1}) adds to the FP64 accumulator:
//     on:  acc += a_prev z_{k-1} + a_cur z_k + a_next z_{k+1}
//     off: nothing (a later launch of the same series adds it).
// A launch may leave its update to the next one or two launches, whose
// epilogues still hold z_{k-1} and z_k: two or three terms then cost one
// read-modify-write of acc.
struct AccUpdate {
  double a_prev, a_cur, a_next;
  int on;
};

// ---- single-vector path (W = 1) ----
// src: caller vector (p or x0) or the plan's own residual; b = scale * src.
hipError_t init_w1(const cpaa_plan_s* pl, Workspace& ws, const double* src, double scale,
                   bool add, bool store_b, bool series, hipStream_t st);
hipError_t load_x0_w1(const cpaa_plan_s* pl, Workspace& ws, const double* x0, hipStream_t st);
hipError_t term_w1(const cpaa_plan_s* pl, Workspace& ws, int cur, int prev, int next,
                   bool first, const AccUpdate& au, double* cert_slot, const int* done,
                   hipStream_t st);
hipError_t check_series(const cpaa_plan_s* pl, Workspace& ws, const double* cert_slot,
                        double scale, double target, int term_index, hipStream_t st);
// r = b - (I - cP) x for x = D acc, with its statistics; where the residual's
// pass can (hub-sliced plans) it also writes x (non-null) at the caller's
// labels and sets *wrote_x
hipError_t residual_w1(const cpaa_plan_s* pl, Workspace& ws, hipStream_t st,
                       double* x = nullptr, bool* wrote_x = nullptr);
hipError_t finalize_w1(const cpaa_plan_s* pl, Workspace& ws, double* x, double scale,
                       hipStream_t st);
// Dropped (edgeless) vertices of a drop_isolated plan: their share of the
// right-hand side's statistics ([0] sum, [3] sum over dropped vertices, [4]
// negative and [5] non-finite counts), and their results x_v = scale * p_v.
hipError_t dropped_stats(const cpaa_plan_s* pl, Workspace& ws, const double* src,
                         hipStream_t st);
hipError_t dropped_out(const cpaa_plan_s* pl, const double* src, double scale, double* x,
                       hipStream_t st);

// ---- directed graphs: the power method in x-space (kernels_w1.hip) ----
// acc (+)= x_0 = scale * src, z_0 = D_out^+ x_0, dangling mass of x_0 into
// dang[0]; b = (1-c) src when store_b.  Statistics as init_w1's ([0], [4], [5]).
hipError_t init_dir(const cpaa_plan_s* pl, Workspace& ws, const double* src, double scale,
                    bool add, bool store_b, hipStream_t st);
hipError_t term_dir(const cpaa_plan_s* pl, Workspace& ws, int cur, int prev, int next,
                    bool first, const AccUpdate& au, double* cert_slot, const int* done,
                    hipStream_t st);
hipError_t residual_dir(const cpaa_plan_s* pl, Workspace& ws, hipStream_t st);
hipError_t finalize_dir(const cpaa_plan_s* pl, Workspace& ws, double* x, double scale,
                        hipStream_t st);

// ---- tiled path (W right-hand sides per tile) ----
hipError_t init_tile(const cpaa_plan_s* pl, Workspace& ws, const double* P, int64_t ldp, int B,
                     double scale, bool add, bool store_b, bool series, hipStream_t st);
hipError_t init_tile_from_r(const cpaa_plan_s* pl, Workspace& ws, const int* active,
                            const int* plain, hipStream_t st);
hipError_t load_x0_tile(const cpaa_plan_s* pl, Workspace& ws, const double* X0, int64_t ldx0,
                        int B, hipStream_t st);
hipError_t term_tile(const cpaa_plan_s* pl, Workspace& ws, int cur, int prev, int next,
                     bool first, const AccUpdate& au, double* cert_slot, const int* done,
                     hipStream_t st);
hipError_t residual_tile(const cpaa_plan_s* pl, Workspace& ws, const int* active, hipStream_t st);
hipError_t finalize_tile(const cpaa_plan_s* pl, Workspace& ws, double* X, int64_t ldx, int B,
                         const double* col_scale, hipStream_t st);
hipError_t init_done(Workspace& ws, const int* active, hipStream_t st);

// ---- multi-graph path (graphs.hip) ----
cpaa_status build_graph_state(cpaa_plan_s* pl, const int32_t* rp, const int32_t* ci,
                              const int32_t* gp);
void free_graph_state(cpaa_plan_s* pl);
cpaa_status solve_graphs_impl(cpaa_plan_s* pl, const double* p, double tol, double* x,
                              cpaa_report* reps, hipStream_t st);

// ---- host helpers (solve.hip) ----
cpaa_status ensure_workspace(cpaa_plan_s* pl, Workspace& ws, int W, int tiles);
void select_map(cpaa_plan_s* pl, size_t i);
void free_workspace(Workspace& ws);
double series_tail(const cpaa_plan_s* pl, int M);
int apriori_terms(const cpaa_plan_s* pl, double norm_dinv_half_b, double target);
int mass_rule_terms(const cpaa_plan_s* pl, double target);

}  // namespace cpaa
