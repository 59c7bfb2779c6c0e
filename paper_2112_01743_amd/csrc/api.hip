// Plan construction, validation and the small C entry points.
//
// The plan is the host-side "graph builder": it checks that the input is the
// symmetric pattern of an undirected graph with every degree positive (the
// setting of Sec. 2.1, where P = A D^{-1} and I - cP is invertible), computes
// degrees and vol, cuts the CSR into workgroup work items, tabulates the
// Chebyshev coefficients c_k = 2 beta^k / sqrt(1-c^2) (Prop. 1) and uploads
// the pattern to the device.
#include <algorithm>
#include <cfloat>
#include <thread>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace cpaa {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

namespace {

template <typename T>
cpaa_status dev_alloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    set_error(std::string("device allocation of ") + std::to_string(count * sizeof(T)) +
              " bytes failed: " + hipGetErrorString(e));
    (void)hipGetLastError();
    return CPAA_ENOMEM;
  }
  return CPAA_OK;
}

template <typename T>
cpaa_status dev_upload(T** p, const T* src, size_t count) {
  cpaa_status s = dev_alloc(p, count);
  if (s != CPAA_OK) return s;
  if (count) CPAA_HIP(hipMemcpy(*p, src, count * sizeof(T), hipMemcpyHostToDevice));
  return CPAA_OK;
}

cpaa_status validate_pattern(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* ci,
                             bool check_symmetry, bool allow_empty_rows = false) {
  if (rp[0] != 0 || static_cast<int64_t>(rp[n]) != nnz) {
    set_error("row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
    return CPAA_EPATTERN;
  }
  for (int32_t u = 0; u < n; ++u) {
    const int32_t a = rp[u], e = rp[u + 1];
    if (e < a) {
      set_error("row_ptr is not monotone at row " + std::to_string(u));
      return CPAA_EPATTERN;
    }
    if (e == a && !allow_empty_rows) {
      set_error("vertex " + std::to_string(u) + " is isolated (degree 0)");
      return CPAA_EISOLATED;
    }
    int32_t last = -1;
    for (int32_t j = a; j < e; ++j) {
      const int32_t v = ci[j];
      if (v < 0 || v >= n) {
        set_error("column index out of range in row " + std::to_string(u));
        return CPAA_EPATTERN;
      }
      if (v == u) {
        set_error("self loop at vertex " + std::to_string(u));
        return CPAA_ESELFLOOP;
      }
      if (v <= last) {
        set_error("columns of row " + std::to_string(u) + " are unsorted or duplicated");
        return CPAA_EPATTERN;
      }
      last = v;
    }
  }
  if (!check_symmetry) return CPAA_OK;
  // The transpose built by a counting pass over rows in increasing order has
  // sorted rows; a symmetric pattern equals its transpose entry for entry.
  std::vector<int64_t> cursor(rp, rp + n);
  std::vector<int32_t> tcol(static_cast<size_t>(nnz));
  for (int32_t u = 0; u < n; ++u) {
    for (int32_t j = rp[u]; j < rp[u + 1]; ++j) {
      const int32_t v = ci[j];
      const int64_t pos = cursor[v]++;
      if (pos >= rp[v + 1]) {
        set_error("adjacency pattern is not symmetric (row " + std::to_string(v) +
                  " receives more entries than it stores)");
        return CPAA_ENOTSYM;
      }
      tcol[pos] = u;
    }
  }
  for (int64_t j = 0; j < nnz; ++j) {
    if (tcol[j] != ci[j]) {
      set_error("adjacency pattern is not symmetric");
      return CPAA_ENOTSYM;
    }
  }
  return CPAA_OK;
}

// Work items of the single-vector kernels (see WorkItem).
void build_items(int32_t n, const int32_t* rp, int npt, std::vector<WorkItem>& items,
                 std::vector<int>& split_nchunks) {
  const int cap = kWG * npt;
  items.clear();
  split_nchunks.clear();
  int32_t r = 0;
  while (r < n) {
    const int d = rp[r + 1] - rp[r];
    if (d > cap) {
      const int slot = static_cast<int>(split_nchunks.size());
      const int nch = (d + cap - 1) / cap;
      for (int c = 0; c < nch; ++c) {
        const int a = rp[r] + c * cap;
        items.push_back({r, -(slot + 1), a, std::min(a + cap, rp[r + 1])});
      }
      split_nchunks.push_back(nch);
      ++r;
      continue;
    }
    const bool is_long = d > kLongRow;
    const int32_t r0 = r;
    int tot = 0;
    while (r < n && (r - r0) < kWG * 4) {
      const int dr = rp[r + 1] - rp[r];
      if (dr > cap || (dr > kLongRow) != is_long || tot + dr > cap) break;
      tot += dr;
      ++r;
    }
    items.push_back({r0, r, rp[r0], rp[r]});
  }
}

// Work items of the tiled kernels, one per wavefront: groups of short rows with
// at most kTileShortNnz entries, or chunks of kTileChunkNnz entries of a row
// longer than kTileLongDeg.
void build_tile_items(int32_t n, const int32_t* rp, std::vector<WorkItem>& items,
                      std::vector<int>& split_nchunks) {
  items.clear();
  split_nchunks.clear();
  int32_t r = 0;
  while (r < n) {
    const int d = rp[r + 1] - rp[r];
    if (d > kTileLongDeg) {
      const int slot = static_cast<int>(split_nchunks.size());
      const int nch = (d + kTileChunkNnz - 1) / kTileChunkNnz;
      for (int c = 0; c < nch; ++c) {
        const int a = rp[r] + c * kTileChunkNnz;
        items.push_back({r, -(slot + 1), a, std::min(a + kTileChunkNnz, rp[r + 1])});
      }
      split_nchunks.push_back(nch);
      ++r;
      continue;
    }
    const int32_t r0 = r;
    int tot = 0;
    while (r < n && (r - r0) < 64) {
      const int dr = rp[r + 1] - rp[r];
      if (dr > kTileLongDeg || (r > r0 && tot + dr > kTileShortNnz)) break;
      tot += dr;
      ++r;
    }
    items.push_back({r0, r, rp[r0], rp[r]});
  }
}

// Run body(i) for i in [0, count) on up to 16 host threads.
template <typename F>
void parallel_for(int64_t count, F body) {
  const int64_t nt = std::max<int64_t>(
      1, std::min<int64_t>({16, (int64_t)std::thread::hardware_concurrency(), count}));
  std::vector<std::thread> pool;
  auto run = [&](int64_t t) {
    for (int64_t i = t * count / nt; i < (t + 1) * count / nt; ++i) body(i);
  };
  for (int64_t t = 1; t < nt; ++t) pool.emplace_back(run, t);
  run(0);
  for (std::thread& th : pool) th.join();
}

// The CSR of the same graph under new labels: perm[new] = old; columns sorted.
void relabel_csr(int32_t n, const int32_t* rp, const int32_t* ci, const std::vector<int32_t>& perm,
                 std::vector<int32_t>& rp2, std::vector<int32_t>& ci2) {
  std::vector<int32_t> new_of(n);
  for (int32_t u = 0; u < n; ++u) new_of[perm[u]] = u;
  rp2.assign(static_cast<size_t>(n) + 1, 0);
  for (int32_t u = 0; u < n; ++u) rp2[u + 1] = rp2[u] + (rp[perm[u] + 1] - rp[perm[u]]);
  ci2.resize(static_cast<size_t>(rp2[n]));
  parallel_for(n, [&](int64_t u) {
    const int32_t v = perm[u];
    int32_t* dst = ci2.data() + rp2[u];
    for (int32_t j = rp[v]; j < rp[v + 1]; ++j) *dst++ = new_of[ci[j]];
    std::sort(ci2.data() + rp2[u], dst);
  });
}

// Mean distance |u - v| between the labels of a stored entry's row and column:
// how far apart in the vector the gathers of neighbouring rows fall.
double mean_span(int32_t n, const int32_t* rp, const int32_t* ci) {
  double sum = 0.0;
  for (int32_t u = 0; u < n; ++u)
    for (int32_t j = rp[u]; j < rp[u + 1]; ++j) sum += std::abs(static_cast<double>(ci[j] - u));
  return rp[n] > 0 ? sum / rp[n] : 0.0;
}

// Reverse Cuthill-McKee order, perm[new] = old (Cuthill and McKee 1969, reversed
// as George proposed): per connected component a breadth-first search from a
// pseudo-peripheral vertex (George and Liu's iteration: from a vertex of least
// degree, restart from a least-degree vertex of the deepest level while the
// depth grows) that appends each vertex's unvisited neighbours in increasing
// degree; the whole sequence is then reversed.  Neighbouring vertices get
// nearby labels on mesh-like graphs, so a term's gathers stay local.
void rcm_order(int32_t n, const int32_t* rp, const int32_t* ci, std::vector<int32_t>& perm) {
  auto deg = [&](int32_t v) { return rp[v + 1] - rp[v]; };
  std::vector<int32_t> by_deg(n);
  for (int32_t v = 0; v < n; ++v) by_deg[v] = v;
  std::stable_sort(by_deg.begin(), by_deg.end(),
                   [&](int32_t a, int32_t b) { return deg(a) < deg(b); });
  std::vector<char> placed(n, 0);
  std::vector<int32_t> dist(n, -1), seen;
  std::vector<int32_t> order, nb;
  order.reserve(n);
  for (int32_t s0 : by_deg) {
    if (placed[s0]) continue;
    int32_t root = s0;
    int depth = -1;
    for (int it = 0; it < 8; ++it) {
      // levels of a breadth-first search from root; every vertex of the
      // component is reached (the component holds no placed vertex yet)
      seen.clear();
      seen.push_back(root);
      dist[root] = 0;
      for (size_t h = 0; h < seen.size(); ++h) {
        const int32_t v = seen[h];
        for (int32_t j = rp[v]; j < rp[v + 1]; ++j)
          if (dist[ci[j]] < 0) {
            dist[ci[j]] = dist[v] + 1;
            seen.push_back(ci[j]);
          }
      }
      const int d = dist[seen.back()];
      int32_t far = seen.back();
      for (size_t h = seen.size(); h-- > 0 && dist[seen[h]] == d;)
        if (deg(seen[h]) < deg(far)) far = seen[h];
      for (int32_t v : seen) dist[v] = -1;
      if (d <= depth) break;
      depth = d;
      root = far;
    }
    size_t head = order.size();
    order.push_back(root);
    placed[root] = 1;
    while (head < order.size()) {
      const int32_t v = order[head++];
      nb.clear();
      for (int32_t j = rp[v]; j < rp[v + 1]; ++j)
        if (!placed[ci[j]]) {
          placed[ci[j]] = 1;
          nb.push_back(ci[j]);
        }
      std::stable_sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) { return deg(a) < deg(b); });
      order.insert(order.end(), nb.begin(), nb.end());
    }
  }
  perm.assign(order.rbegin(), order.rend());
}

// Smallest eigenvalue of P, estimated by m steps of the Lanczos iteration on
// the symmetric S = D^{-1/2} A D^{-1/2} (similar to P, so the same spectrum)
// from a fixed pseudo-random start: the smallest eigenvalue of the Lanczos
// tridiagonal matrix, found by bisection on its Sturm sequence.  A Ritz value
// is never below the true smallest eigenvalue and approaches it from above.
double lanczos_lambda_min(int32_t n, const int32_t* rp, const int32_t* ci, int m) {
  std::vector<double> isd(n), q(n), qp(n, 0.0), w(n);
  for (int32_t u = 0; u < n; ++u) isd[u] = 1.0 / std::sqrt(static_cast<double>(rp[u + 1] - rp[u]));
  uint64_t x = 0x9E3779B97F4A7C15ull;             // xorshift64 start vector
  double nrm = 0.0;
  for (int32_t u = 0; u < n; ++u) {
    x ^= x << 13;
    x ^= x >> 7;
    x ^= x << 17;
    q[u] = static_cast<double>(x >> 11) * 0x1p-53 - 0.5;
    nrm += q[u] * q[u];
  }
  for (double& v : q) v /= std::sqrt(nrm);
  std::vector<double> al, be;
  double bprev = 0.0;
  for (int j = 0; j < m; ++j) {
    parallel_for(n, [&](int64_t u) {
      double t = 0.0;
      for (int32_t k = rp[u]; k < rp[u + 1]; ++k) t += isd[ci[k]] * q[ci[k]];
      w[u] = isd[u] * t;
    });
    double a = 0.0;
    for (int32_t u = 0; u < n; ++u) a += w[u] * q[u];
    double b2 = 0.0;
    for (int32_t u = 0; u < n; ++u) {
      w[u] -= a * q[u] + bprev * qp[u];
      b2 += w[u] * w[u];
    }
    al.push_back(a);
    const double b = std::sqrt(b2);
    if (b < 1e-12 || j + 1 == m) break;
    be.push_back(b);
    for (int32_t u = 0; u < n; ++u) {
      qp[u] = q[u];
      q[u] = w[u] / b;
    }
    bprev = b;
  }
  // number of eigenvalues of the tridiagonal matrix below t (Sturm sequence)
  auto below = [&](double t) {
    int cnt = 0;
    double d = 1.0;
    for (size_t i = 0; i < al.size(); ++i) {
      const double off = i ? be[i - 1] * be[i - 1] : 0.0;
      d = al[i] - t - (i ? off / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0.0) ++cnt;
    }
    return cnt;
  };
  double lo = -1.5, hi = 1.5;
  for (int it = 0; it < 100; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (below(mid) >= 1) hi = mid; else lo = mid;
  }
  return hi;
}

// Labelling of the column-sliced path: vertices ranked by degree (descending,
// ties by label) and dealt round-robin, in groups of 8 ranks, into kSlices
// slices, slice s taking the contiguous labels [slice_off[s], slice_off[s+1]).
// Every slice gets n/8 vertices and about vol/8 stored entries as columns.  Returns the relabelled
// CSR (rows and columns in new labels, columns sorted) and perm[new] = old.
void slice_relabel(int32_t n, const int32_t* rp, const int32_t* ci, std::vector<int32_t>& rp2,
                   std::vector<int32_t>& ci2, std::vector<int32_t>& perm,
                   int slice_off[kSlices + 1]) {
  std::vector<int32_t> order(n);
  for (int32_t v = 0; v < n; ++v) order[v] = v;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return rp[a + 1] - rp[a] > rp[b + 1] - rp[b];
  });
  // ranks are dealt in groups of kDeal (8 doubles = one 64-byte line), so
  // vertices that are neighbours in the caller's order and in rank stay
  // neighbours in a slice (cheap gathers and scatters of p and x)
  constexpr int32_t kDeal = 8;
  auto slice_of = [&](int32_t r) { return (r / kDeal) % kSlices; };
  int32_t count[kSlices] = {};
  for (int32_t r = 0; r < n; ++r) ++count[slice_of(r)];
  slice_off[0] = 0;
  for (int sl = 0; sl < kSlices; ++sl) slice_off[sl + 1] = slice_off[sl] + count[sl];
  perm.assign(n, 0);
  for (int32_t r = 0; r < n; ++r)
    perm[slice_off[slice_of(r)] + (r / (kDeal * kSlices)) * kDeal + r % kDeal] = order[r];
  relabel_csr(n, rp, ci, perm, rp2, ci2);
}

// Work items and packed entries of the column-sliced term (relabelled CSR).
// Per slice the items cover every row (rows without entries in the slice
// still get their zero partial written): consecutive rows with at most
// kWG * kSliceNpt entries and 2^row_bits rows per item; a row with more entries
// in one slice than an item holds is cut into split chunks (plain local
// columns, nnz1 = physical end).  Multi-row items store their entries in the
// transposed per-wavefront layout described below; nnz0 is the physical start
// and nnz1 - nnz0 the number of entries (the layout pads each wavefront's
// share to a multiple of 64 with kSliceNone).
bool build_sliced(int32_t n, const std::vector<int32_t>& rp2, const std::vector<int32_t>& ci2,
                  const int slice_off[kSlices + 1], int row_bits, std::vector<uint32_t>& entries,
                  std::vector<WorkItem>& items, std::vector<int>& split_nchunks,
                  int item_off[kSlices + 1]) {
  const int cap = kWG * kSliceNpt;
  std::vector<std::vector<uint32_t>> ent(kSlices);
  std::vector<std::vector<WorkItem>> its(kSlices);
  std::vector<std::vector<int>> nch(kSlices);
  parallel_for(kSlices, [&](int64_t sl) {
    const int32_t lo = slice_off[sl], hi = slice_off[sl + 1];
    std::vector<int32_t> beg(n), len(n);
    for (int32_t u = 0; u < n; ++u) {
      const int32_t* a = ci2.data() + rp2[u];
      const int32_t* b = ci2.data() + rp2[u + 1];
      const int32_t* x = std::lower_bound(a, b, lo);
      const int32_t* y = std::lower_bound(x, b, hi);
      beg[u] = static_cast<int32_t>(x - ci2.data());
      len[u] = static_cast<int32_t>(y - x);
    }
    std::vector<uint32_t>& E = ent[sl];
    std::vector<WorkItem>& I = its[sl];
    std::vector<uint32_t> logical;
    int32_t r = 0;
    while (r < n) {
      if (len[r] > cap) {
        const int slot = static_cast<int>(nch[sl].size());
        const int chunks = (len[r] + cap - 1) / cap;
        for (int c = 0; c < chunks; ++c) {
          const int e0 = static_cast<int>(E.size());
          const int a = beg[r] + c * cap, b = std::min(a + cap, beg[r] + len[r]);
          for (int j = a; j < b; ++j) E.push_back(static_cast<uint32_t>(ci2[j] - lo));
          I.push_back({r, -(slot + 1), e0, static_cast<int>(E.size())});
        }
        nch[sl].push_back(chunks);
        ++r;
        continue;
      }
      const int32_t r0 = r;
      logical.clear();
      while (r < n && r - r0 < (1 << row_bits) && len[r] <= cap &&
             static_cast<int>(logical.size()) + len[r] <= cap) {
        for (int j = beg[r]; j < beg[r] + len[r]; ++j)
          logical.push_back((static_cast<uint32_t>(ci2[j] - lo) << row_bits) |
                            static_cast<uint32_t>(r - r0));
        ++r;
      }
      // Wavefront w takes logical entries [w*64*kSliceNpt, ...), lane l a
      // contiguous run of RL = ceil(len/64) of them, stored transposed
      // (run element i of lane l at i*64 + l) so the loads stay coalesced.
      const int e0 = static_cast<int>(E.size());
      const int L = static_cast<int>(logical.size());
      for (int q0 = 0; q0 < L; q0 += 64 * kSliceNpt) {
        const int Lw = std::min(64 * kSliceNpt, L - q0);
        const int RL = (Lw + 63) / 64;
        const size_t pb = E.size();
        E.resize(pb + static_cast<size_t>(64) * RL, kSliceNone);
        for (int q = 0; q < Lw; ++q) E[pb + (q % RL) * 64 + q / RL] = logical[q0 + q];
      }
      I.push_back({r0, r, e0, e0 + L});   // nnz1 - nnz0 = logical length
    }
  });
  // int offsets below: the padded total must fit (every local offset is smaller)
  int64_t etot = 0;
  for (int sl = 0; sl < kSlices; ++sl) etot += static_cast<int64_t>(ent[sl].size());
  if (etot > kSliceEntryLimit) return false;
  entries.clear();
  items.clear();
  split_nchunks.clear();
  item_off[0] = 0;
  for (int sl = 0; sl < kSlices; ++sl) {
    const int ebase = static_cast<int>(entries.size());
    const int sbase = static_cast<int>(split_nchunks.size());
    for (WorkItem it : its[sl]) {
      it.nnz0 += ebase;
      it.nnz1 += ebase;
      if (it.row1 < 0) it.row1 -= sbase;
      items.push_back(it);
    }
    entries.insert(entries.end(), ent[sl].begin(), ent[sl].end());
    split_nchunks.insert(split_nchunks.end(), nch[sl].begin(), nch[sl].end());
    item_off[sl + 1] = static_cast<int>(items.size());
  }
  return true;
}

// Host image of a HubMap (internal.h).
struct HubHost {
  std::vector<uint32_t> entries;
  std::vector<HubItem> items;
  int item_off[kSlices + 1] = {};
  int pofs[kSlices + 1] = {};
  std::vector<uint8_t> mask;
  std::vector<int32_t> base;
  std::vector<int> chunk_long, long_first, long_nch, long_out;
  int cfg = 0;   // launch shape (kHubShapes index) the map was built for
};

// Packed entries, wave items, compact partial indices and long-row chunks of
// the hub-sliced term (layout in internal.h), from the relabelled CSR
// (columns sorted); a wave item holds at most row_cap (<= kHubRows) present
// rows.  Returns false when the entry array (with its run padding) or the
// partial array would outgrow int offsets; h is then unusable.
bool build_hub_sliced(int32_t n, const std::vector<int32_t>& rp2, const std::vector<int32_t>& ci2,
                      const int slice_off[kSlices + 1], int row_cap, HubHost& h) {
  struct LocalItem {
    int64_t j0, e0;
    int len, rows;
  };
  struct SliceOut {
    std::vector<uint32_t> E;
    std::vector<LocalItem> I;
    std::vector<uint8_t> present;
    int64_t P = 0;
    std::vector<int64_t> lj;      // long rows: compact row
    std::vector<int> lfirst, lnch;
  };
  std::vector<SliceOut> so(kSlices);
  const int64_t nblk = (static_cast<int64_t>(n) + 63) / 64;
  h.base.assign(static_cast<size_t>(nblk) * kSlices, 0);
  parallel_for(kSlices, [&](int64_t sl) {
    SliceOut& o = so[sl];
    const int32_t lo = slice_off[sl], hi = slice_off[sl + 1];
    o.present.assign(n, 0);
    std::vector<uint32_t> logical;
    int cur_rows = 0, chunks = 0;
    int64_t cur_j0 = 0, j = 0;
    auto flush = [&]() {
      if (cur_rows == 0) return;
      const int L = static_cast<int>(logical.size());
      const int RL = hub_run_length(L);
      o.E.resize((o.E.size() + 3) & ~size_t(3), kSliceNone);   // 16-byte aligned item
      const size_t pb = o.E.size();
      o.E.resize(pb + static_cast<size_t>(64) * RL, kSliceNone);
      for (int q = 0; q < L; ++q) o.E[pb + hub_slot(q / RL, q % RL)] = logical[q];
      o.I.push_back({cur_j0, static_cast<int64_t>(pb), L, cur_rows});
      logical.clear();
      cur_rows = 0;
    };
    for (int32_t u = 0; u < n; ++u) {
      if ((u & 63) == 0) h.base[static_cast<size_t>(u >> 6) * kSlices + sl] = static_cast<int32_t>(j);
      const int32_t* a = ci2.data() + rp2[u];
      const int32_t* b = ci2.data() + rp2[u + 1];
      const int32_t* x = std::lower_bound(a, b, lo);
      const int32_t* y = std::lower_bound(x, b, hi);
      const int len = static_cast<int>(y - x);
      if (len == 0) continue;
      o.present[u] = 1;
      if (len > kHubItemCap) {
        flush();
        const int nch = (len + kHubItemCap - 1) / kHubItemCap;
        o.lj.push_back(j);
        o.lfirst.push_back(chunks);
        o.lnch.push_back(nch);
        for (int c = 0; c < nch; ++c) {
          const int cl = std::min(kHubItemCap, len - c * kHubItemCap);
          const size_t pb = o.E.size();
          for (int t = 0; t < cl; ++t)
            o.E.push_back(static_cast<uint32_t>(x[c * kHubItemCap + t] - lo));
          o.I.push_back({j, static_cast<int64_t>(pb), cl, -(chunks + 1)});
          ++chunks;
        }
        ++j;
        continue;
      }
      if (cur_rows > 0 &&
          (static_cast<int>(logical.size()) + len > kHubItemCap || cur_rows == row_cap))
        flush();
      if (cur_rows == 0) cur_j0 = j;
      for (const int32_t* q = x; q < y; ++q)
        logical.push_back((static_cast<uint32_t>(*q - lo) << kHubRowBits) |
                          static_cast<uint32_t>(cur_rows));
      ++cur_rows;
      ++j;
    }
    flush();
    o.P = j;
  });
  int64_t etot = 0, ptot = 0, itot = 0;
  for (const SliceOut& o : so) {
    etot += static_cast<int64_t>(o.E.size());
    ptot += o.P;
    itot += static_cast<int64_t>(o.I.size());
  }
  if (etot > kSliceEntryLimit || ptot > INT32_MAX || itot > INT32_MAX) return false;
  h.entries.clear();
  h.entries.reserve(static_cast<size_t>(etot));
  h.items.clear();
  h.items.reserve(static_cast<size_t>(itot));
  int64_t ebase = 0, pbase = 0;
  int cbase = 0, lbase = 0;
  for (int sl = 0; sl < kSlices; ++sl) {
    const SliceOut& o = so[sl];
    h.item_off[sl] = static_cast<int>(h.items.size());
    h.pofs[sl] = static_cast<int>(pbase);
    for (const LocalItem& it : o.I)
      h.items.push_back({static_cast<int>(it.j0), static_cast<int>(it.e0 + ebase), it.len,
                         it.rows < 0 ? it.rows - cbase : it.rows});
    for (size_t q = 0; q < o.lj.size(); ++q) {
      h.long_first.push_back(o.lfirst[q] + cbase);
      h.long_nch.push_back(o.lnch[q]);
      h.long_out.push_back(static_cast<int>(pbase + o.lj[q]));
      for (int c = 0; c < o.lnch[q]; ++c) h.chunk_long.push_back(lbase + static_cast<int>(q));
    }
    cbase += o.lnch.empty() ? 0 : o.lfirst.back() + o.lnch.back();
    lbase += static_cast<int>(o.lj.size());
    h.entries.insert(h.entries.end(), o.E.begin(), o.E.end());
    ebase += static_cast<int64_t>(o.E.size());
    pbase += o.P;
  }
  h.item_off[kSlices] = static_cast<int>(h.items.size());
  h.pofs[kSlices] = static_cast<int>(pbase);
  h.mask.assign(n, 0);
  for (int sl = 0; sl < kSlices; ++sl)
    for (int32_t u = 0; u < n; ++u) h.mask[u] |= static_cast<uint8_t>(so[sl].present[u] << sl);
  return true;
}

// Structural check of a hub map against what the kernels index: every item's
// run layout inside the entry array, packed rows below the item's row count
// and local columns inside the slice, partial indices inside the slice's
// range, the block bases consistent with the masks.  Runs once per plan on
// the host (linear in the entries).
bool check_hub_map(int32_t n, const int slice_off[kSlices + 1], const HubHost& h,
                   std::string& why) {
  const size_t ne = h.entries.size();
  for (int sl = 0; sl < kSlices; ++sl) {
    const uint32_t nsl = static_cast<uint32_t>(slice_off[sl + 1] - slice_off[sl]);
    const int64_t P = static_cast<int64_t>(h.pofs[sl + 1]) - h.pofs[sl];
    for (int k = h.item_off[sl]; k < h.item_off[sl + 1]; ++k) {
      const HubItem& it = h.items[k];
      if (it.len <= 0 || it.len > kHubItemCap || it.e0 < 0 || it.j0 < 0) {
        why = "item bounds";
        return false;
      }
      if (it.rows < 0) {
        const int slot = -(it.rows + 1);
        if (slot >= static_cast<int>(h.chunk_long.size()) ||
            static_cast<size_t>(it.e0) + it.len > ne || it.j0 >= P) {
          why = "chunk item";
          return false;
        }
        for (int t = 0; t < it.len; ++t)
          if (h.entries[it.e0 + t] >= nsl) {
            why = "chunk column";
            return false;
          }
        continue;
      }
      const int RL = hub_run_length(it.len);
      if (it.rows > kHubRows || it.rows > it.len || it.j0 + static_cast<int64_t>(it.rows) > P ||
          static_cast<size_t>(it.e0) + static_cast<size_t>(64) * RL > ne || (it.e0 & 3) != 0 ||
          RL > kHubNpt) {
        why = "item rows or run layout";
        return false;
      }
      // logical entry q is element q % RL of lane q / RL; rows ascend over q
      // (the kernel's cross-lane scan relies on it) and every row appears
      int prev = 0;
      for (int q = 0; q < it.len; ++q) {
        const uint32_t e = h.entries[it.e0 + hub_slot(q / RL, q % RL)];
        const int r = static_cast<int>(e & ((1u << kHubRowBits) - 1u));
        if (e == kSliceNone || (e >> kHubRowBits) >= nsl || r >= it.rows || r < prev ||
            r > prev + 1 || (q == 0 && r != 0)) {
          why = "packed entry";
          return false;
        }
        prev = r;
      }
      if (prev != it.rows - 1) {
        why = "rows of an item";
        return false;
      }
      for (int l = 0; l < 64; ++l)
        for (int i = std::max(0, std::min(RL, it.len - l * RL)); i < RL; ++i)
          if (h.entries[it.e0 + hub_slot(l, i)] != kSliceNone) {
            why = "padding";
            return false;
          }
    }
  }
  for (size_t q = 0; q < h.long_out.size(); ++q)
    if (h.long_out[q] < 0 || h.long_out[q] >= h.pofs[kSlices] || h.long_nch[q] < 2 ||
        h.long_first[q] + h.long_nch[q] > static_cast<int>(h.chunk_long.size())) {
      why = "long row";
      return false;
    }
  std::vector<int64_t> cnt(kSlices, 0);
  for (int32_t u = 0; u < n; ++u) {
    for (int sl = 0; sl < kSlices; ++sl) {
      if ((u & 63) == 0 && h.base[static_cast<size_t>(u >> 6) * kSlices + sl] != cnt[sl]) {
        why = "block base";
        return false;
      }
      cnt[sl] += (h.mask[u] >> sl) & 1;
    }
  }
  for (int sl = 0; sl < kSlices; ++sl)
    if (cnt[sl] != static_cast<int64_t>(h.pofs[sl + 1]) - h.pofs[sl]) {
      why = "present rows";
      return false;
    }
  return true;
}

}  // namespace
}  // namespace cpaa

namespace cpaa {
void select_map(cpaa_plan_s* pl, size_t i) {
  const WorkMap& m = pl->maps[i];
  pl->npt = m.npt;
  pl->d_items = m.d_items;
  pl->n_items = m.n_items;
  pl->n_split_rows = m.n_split_rows;
  pl->d_split_nchunks = m.d_split_nchunks;
}
}  // namespace cpaa

using namespace cpaa;

extern "C" {

const char* cpaa_last_error(void) { return g_last_error.c_str(); }

void cpaa_default_opts(cpaa_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->k_max = 0;
  o->max_refine = 2;
  o->normalize = 0;
  o->nnz_per_thread = 0;
  o->tile_w = 0;
  o->validate = 1;
  o->io_device = 1;
  o->time_kernels = 0;
  o->xcd_remap = -1;
  o->autotune = 0;
  o->column_slices = 0;
  o->locality_order = 0;
  o->spectral_interval = 0;
  o->directed = 0;
  o->slice_shape = 0;
  o->rows_per_wave = 0;
  o->fp64_recurrence = 0;
  o->deterministic = 0;
  o->drop_isolated = 0;
}

void cpaa_plan_destroy(cpaa_plan_t pl) {
  if (!pl) return;
  free_workspace(pl->ws1);
  free_workspace(pl->wst);
  free_workspace(pl->wsg);
  free_graph_state(pl);
  for (WorkMap& m : pl->maps) {
    if (m.d_items) (void)hipFree(m.d_items);
    if (m.d_split_nchunks) (void)hipFree(m.d_split_nchunks);
  }
  if (pl->reordered) {
    void* sp[] = {pl->d_rp_w1, pl->d_ci_w1, pl->slc.d_entries, pl->slc.d_items,
                  pl->slc.d_split_nchunks};
    for (void* p : sp)
      if (p) (void)hipFree(p);
  }
  if (pl->d_perm) (void)hipFree(pl->d_perm);
  if (pl->d_dropped) (void)hipFree(pl->d_dropped);
  {
    HubMap& hm = pl->hub;
    void* hp[] = {hm.d_entries, hm.d_items, hm.d_mask, hm.d_base, hm.d_chunk_long,
                  hm.d_long_first, hm.d_long_nch, hm.d_long_out, hm.d_wround};
    for (void* p : hp)
      if (p) (void)hipFree(p);
  }
  void* ptrs[] = {pl->d_row_ptr, pl->d_col_idx, pl->d_dout, pl->d_titems, pl->d_tsplit_nchunks,
                  pl->d_graph_ptr, pl->d_graph_order, pl->d_queue};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (pl->ev_begin) (void)hipEventDestroy(pl->ev_begin);
  if (pl->ev_end) (void)hipEventDestroy(pl->ev_end);
  for (hipEvent_t e : pl->ev_poll)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : pl->ev_terms) (void)hipEventDestroy(e);
  delete pl;
}

cpaa_status cpaa_plan(const cpaa_csr* g, double c, const cpaa_opts* opts, cpaa_plan_t* out) {
  set_error("");
  if (!g || !out) {
    set_error("cpaa_plan: null argument");
    return CPAA_EINVAL;
  }
  *out = nullptr;
  if (!(c > 0.0 && c < 1.0)) {
    set_error("damping factor c must lie in (0, 1)");
    return CPAA_EINVAL;
  }
  if (g->n <= 0 || g->nnz < 0 || g->nnz >= (int64_t(1) << 31) || !g->row_ptr ||
      (g->nnz > 0 && !g->col_idx)) {
    set_error("bad CSR sizes or null CSR arrays");
    return CPAA_EINVAL;
  }
  cpaa_opts o;
  cpaa_default_opts(&o);
  if (opts) o = *opts;
  if (o.nnz_per_thread != 0 && o.nnz_per_thread != 4 && o.nnz_per_thread != 8 &&
      o.nnz_per_thread != 16 && o.nnz_per_thread != 32) {
    set_error("nnz_per_thread must be 0, 4, 8, 16 or 32");
    return CPAA_EINVAL;
  }
  if (o.tile_w != 0 && o.tile_w != 8 && o.tile_w != 16 && o.tile_w != 32 && o.tile_w != 64) {
    set_error("tile_w must be 0, 8, 16, 32 or 64");
    return CPAA_EINVAL;
  }
  if (o.column_slices != 0 && o.column_slices != 1 && o.column_slices != kSlices) {
    set_error("column_slices must be 0, 1 or 8");
    return CPAA_EINVAL;
  }
  if (o.column_slices == kSlices && (g->num_graphs > 1 || g->n >= kSliceMaxN)) {
    set_error("column slices need one graph with n < 8 (2^21 - 16)");
    return CPAA_EINVAL;
  }
  if (o.rows_per_wave < 0 || o.rows_per_wave > kHubRows) {
    set_error("rows_per_wave must be 0 (auto) or 1-" + std::to_string(kHubRows));
    return CPAA_EINVAL;
  }
  if (o.slice_shape < 0 || o.slice_shape > kHubConfigs + 1) {
    set_error("slice_shape must be 0 (auto) or 1-" + std::to_string(kHubConfigs + 1));
    return CPAA_EINVAL;
  }
  if ((o.fp64_recurrence != 0 && o.fp64_recurrence != 1) ||
      (o.deterministic != 0 && o.deterministic != 1) ||
      (o.drop_isolated != 0 && o.drop_isolated != 1)) {
    set_error("fp64_recurrence, deterministic and drop_isolated must be 0 or 1");
    return CPAA_EINVAL;
  }
  if (o.drop_isolated == 1 && (g->num_graphs > 1 || o.directed != 0)) {
    set_error("drop_isolated needs one undirected graph (directed = 0)");
    return CPAA_EINVAL;
  }
  if (o.fp64_recurrence == 1 && o.column_slices == kSlices) {
    set_error("fp64_recurrence runs in row order (column_slices must be 0 or 1)");
    return CPAA_EINVAL;
  }
  if (o.fp64_recurrence == 1 && o.deterministic == 1) {
    set_error("fp64_recurrence and deterministic cannot be combined");
    return CPAA_EINVAL;
  }
  if (o.deterministic == 1 && (o.column_slices == 1 || o.slice_shape == kHubConfigs + 1)) {
    set_error("deterministic needs the column-sliced term with compact partials "
              "(column_slices 0 or 8, slice_shape 0-" + std::to_string(kHubConfigs) + ")");
    return CPAA_EINVAL;
  }
  if ((o.fp64_recurrence == 1 || o.deterministic == 1) &&
      (g->num_graphs > 1 || o.directed == 1)) {
    set_error("fp64_recurrence and deterministic need one undirected graph");
    return CPAA_EINVAL;
  }
  if (o.spectral_interval != 0 && o.spectral_interval != 1) {
    set_error("spectral_interval must be 0 or 1");
    return CPAA_EINVAL;
  }
  if (o.time_kernels < 0 || o.time_kernels > 2) {
    set_error("time_kernels must be 0, 1 or 2");
    return CPAA_EINVAL;
  }
  if (o.spectral_interval == 1 && g->num_graphs > 1) {
    set_error("spectral_interval needs a single-graph plan");
    return CPAA_EINVAL;
  }
  if (o.directed < 0 || o.directed > 2) {
    set_error("directed must be 0, 1 or 2");
    return CPAA_EINVAL;
  }
  if (o.directed == 1 &&
      (g->num_graphs > 1 || o.locality_order == 2 || o.spectral_interval == 1)) {
    set_error("directed plans need one graph and no RCM or spectral interval");
    return CPAA_EINVAL;
  }
  if (o.locality_order < 0 || o.locality_order > 2) {
    set_error("locality_order must be 0, 1 or 2");
    return CPAA_EINVAL;
  }
  if (o.k_max < 0 || o.max_refine < 0) {
    set_error("k_max and max_refine must be >= 0");
    return CPAA_EINVAL;
  }

  int32_t n = g->n;
  const int64_t nnz = g->nnz;
  std::vector<int32_t> h_rp, h_ci, h_gp;
  const int32_t* rp = g->row_ptr;
  const int32_t* ci = g->col_idx;
  const int num_graphs = g->num_graphs > 1 ? g->num_graphs : 1;
  const int32_t* gp = g->graph_ptr;
  if (num_graphs > 1 && !gp) {
    set_error("num_graphs > 1 needs graph_ptr");
    return CPAA_EINVAL;
  }
  if (g->on_device) {
    h_rp.resize(n + 1);
    h_ci.resize(static_cast<size_t>(nnz));
    CPAA_HIP(hipMemcpy(h_rp.data(), g->row_ptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (nnz)
      CPAA_HIP(hipMemcpy(h_ci.data(), g->col_idx, nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
    rp = h_rp.data();
    ci = h_ci.data();
    if (num_graphs > 1) {
      h_gp.resize(num_graphs + 1);
      CPAA_HIP(hipMemcpy(h_gp.data(), g->graph_ptr, (num_graphs + 1) * sizeof(int32_t),
                         hipMemcpyDeviceToHost));
      gp = h_gp.data();
    }
  }
  bool directed = o.directed == 1;
  if (o.directed == 2) {
    // detect: a pattern that is not symmetric, or has an empty row (a dangling
    // vertex), makes a directed plan
    cpaa_status s = validate_pattern(n, nnz, rp, ci, false, true);
    if (s != CPAA_OK) return s;
    directed = validate_pattern(n, nnz, rp, ci, true, false) != CPAA_OK;
    set_error("");
    if (directed && (g->num_graphs > 1 || o.locality_order == 2 || o.spectral_interval == 1 ||
                     o.fp64_recurrence == 1 || o.deterministic == 1)) {
      set_error("the pattern is directed (not symmetric, or with an empty row); directed plans "
                "need one graph and no RCM, spectral interval, fp64_recurrence or deterministic");
      return CPAA_EINVAL;
    }
  } else if (o.validate) {
    cpaa_status s = validate_pattern(n, nnz, rp, ci, !directed, directed || o.drop_isolated == 1);
    if (s != CPAA_OK) return s;
  } else if (rp[0] != 0 || rp[n] != nnz) {
    set_error("row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
    return CPAA_EPATTERN;
  }
  if (num_graphs > 1) {
    if (gp[0] != 0 || gp[num_graphs] != n) {
      set_error("graph_ptr must start at 0 and end at n");
      return CPAA_EINVAL;
    }
    for (int gi = 0; gi < num_graphs; ++gi) {
      if (gp[gi + 1] <= gp[gi]) {
        set_error("graph_ptr must be strictly increasing");
        return CPAA_EINVAL;
      }
      if (o.validate) {
        for (int32_t u = gp[gi]; u < gp[gi + 1]; ++u)
          for (int32_t j = rp[u]; j < rp[u + 1]; ++j)
            if (ci[j] < gp[gi] || ci[j] >= gp[gi + 1]) {
              set_error("an edge crosses the boundary of graph " + std::to_string(gi));
              return CPAA_EINVAL;
            }
      }
    }
  }
  // Optional per-entry values: Alg. 1 only reads N(u) and the degrees, so a
  // caller's values must be the entries of P = A D^{-1} (Sec. 2.1): the entry
  // of column v is 1/d_v (1/out-degree of v in a directed plan).  They are
  // checked to a few ulps and then not used.
  if (g->values != nullptr && nnz > 0) {
    std::vector<double> h_val;
    const double* val = g->values;
    if (g->on_device) {
      h_val.resize(static_cast<size_t>(nnz));
      CPAA_HIP(hipMemcpy(h_val.data(), g->values, nnz * sizeof(double), hipMemcpyDeviceToHost));
      val = h_val.data();
    }
    std::vector<int32_t> deg_col(n, 0);
    if (directed) {
      for (int64_t j = 0; j < nnz; ++j) ++deg_col[ci[j]];
    } else {
      for (int32_t v = 0; v < n; ++v) deg_col[v] = rp[v + 1] - rp[v];
    }
    for (int64_t j = 0; j < nnz; ++j) {
      const double d = static_cast<double>(deg_col[ci[j]]);
      if (!(std::fabs(val[j] * d - 1.0) <= 4.0 * DBL_EPSILON)) {
        set_error("values[" + std::to_string(static_cast<long long>(j)) +
                  "] is not 1/deg of its column (the entries of P = A D^-1)");
        return CPAA_EINVAL;
      }
    }
  }

  // drop_isolated: the graph without its edgeless vertices, relabelled in order
  // (P has a zero column there and no other vertex depends on them, Sec. 2.1);
  // the solves write x_v = (1-c) p_v for them.
  const int32_t n_caller = n;
  std::vector<int32_t> keep, dropped, red_rp, red_ci;
  if (o.drop_isolated == 1) {
    for (int32_t v = 0; v < n; ++v) (rp[v + 1] > rp[v] ? keep : dropped).push_back(v);
    if (keep.empty()) {
      set_error("drop_isolated: no vertex has an edge");
      return CPAA_EISOLATED;
    }
    if (!dropped.empty()) {
      std::vector<int32_t> nid(n, -1);
      for (size_t i = 0; i < keep.size(); ++i) nid[keep[i]] = static_cast<int32_t>(i);
      red_rp.assign(keep.size() + 1, 0);
      red_ci.resize(static_cast<size_t>(nnz));
      for (size_t i = 0; i < keep.size(); ++i) {
        const int32_t v = keep[i];
        int32_t w = red_rp[i];
        for (int32_t j = rp[v]; j < rp[v + 1]; ++j) red_ci[w++] = nid[ci[j]];   // order kept
        red_rp[i + 1] = w;
      }
      rp = red_rp.data();
      ci = red_ci.data();
      n = static_cast<int32_t>(keep.size());
    }
  }

  cpaa_plan_s* pl = new (std::nothrow) cpaa_plan_s();
  if (!pl) {
    set_error("host allocation failed");
    return CPAA_ENOMEM;
  }
  pl->opts = o;
  pl->n = n;
  pl->n_caller = n_caller;
  pl->n_drop = static_cast<int32_t>(dropped.size());
  pl->nnz = nnz;
  pl->c = c;
  pl->s = std::sqrt(1.0 - c * c);
  pl->beta = (1.0 - pl->s) / c;
  pl->num_graphs = num_graphs;
  (void)hipGetDevice(&pl->device);
  int maxd = 0, mind = INT32_MAX;
  double vol = 0.0;
  for (int32_t u = 0; u < n; ++u) {
    const int d = rp[u + 1] - rp[u];
    maxd = std::max(maxd, d);
    mind = std::min(mind, d);
    vol += d;
  }
  pl->directed = directed;
  if (mind <= 0 && !pl->directed) {
    cpaa_plan_destroy(pl);
    set_error("isolated vertex (degree 0)");
    return CPAA_EISOLATED;
  }
  pl->max_deg = maxd;
  pl->min_deg = mind;
  pl->vol = vol;
  pl->ck.resize(kMaxTerms + 2);
  // Chebyshev expansion on [a, 1] (Sec. 2.2's general interval): a = -1 is the
  // paper's; with spectral_interval, a is a Lanczos estimate of the smallest
  // eigenvalue of P less a margin (no gain below -0.95).  On x = ((1-a)u +
  // (1+a))/2, 1/(1-cx) = (1/A)/(1-c'u), A = 1 - c(1+a)/2, c' = c(1-a)/(2A), so
  // the coefficients are Prop. 1's with c' (beta', s') times 1/A.  The series'
  // certificate identity is algebraic, so a wrong a slows convergence but never
  // the certified result.
  if (o.spectral_interval == 1) {
    const double lam = lanczos_lambda_min(n, rp, ci, 80);
    const double a = lam - 0.02;
    if (a > -0.95) pl->lam_lo = std::min(a, 0.9);
  }
  {
    const double a = pl->lam_lo;
    pl->cheb_A = 1.0 - c * (1.0 + a) / 2.0;
    const double cp = c * (1.0 - a) / (2.0 * pl->cheb_A);
    pl->s = std::sqrt(1.0 - cp * cp);
    pl->beta = (1.0 - pl->s) / cp;
  }
  for (int k = 0; k < kMaxTerms + 2; ++k)
    pl->ck[k] = 2.0 / (pl->cheb_A * pl->s) * std::pow(pl->beta, k);
  pl->pk.assign(kMaxTerms + 2, 1.0 / (1.0 - pl->c));

  // Random gathers into a vector larger than one XCD's L2 are latency bound:
  // large graphs get 32 independent gathers in flight per thread.
  pl->npt = o.nnz_per_thread ? o.nnz_per_thread : (n >= (1 << 20) ? 32 : 16);
  // XCD-contiguous row ranges help lattice-like graphs in the tiled kernel but
  // concentrate the hub rows of power-law graphs on one XCD in the
  // single-vector kernel, so "auto" enables it for tiles only.
  pl->xcd_remap = o.xcd_remap < 0 ? 0 : (o.xcd_remap ? 1 : 0);
  pl->xcd_remap_tile = o.xcd_remap < 0 ? 1 : (o.xcd_remap ? 1 : 0);
  // Column slices keep each XCD's gathers inside one eighth of the vector
  // (its L2); they pay off once the FP32 vector (4n bytes) passes ~3 MB and
  // the degrees are skewed (a lattice's natural order is already local):
  // measured on power-law graphs, 6 % faster at n = 1M, even at 500k.  A
  // directed plan has no RCM alternative, so there a scattered pattern
  // (entries spanning more than 2^14 labels on average) also qualifies.
  const bool big = n >= 3 * (1 << 18) && n < kSliceMaxN;
  pl->fp64 = o.fp64_recurrence == 1;
  pl->deterministic = o.deterministic == 1;
  if (pl->deterministic && n >= kSliceMaxN) {
    cpaa_plan_destroy(pl);
    set_error("deterministic needs the column-sliced term: n < 8 (2^21 - 16)");
    return CPAA_EINVAL;
  }
  pl->sliced = !pl->fp64 &&
               (o.column_slices == kSlices || pl->deterministic ||
                (o.column_slices == 0 && num_graphs == 1 && big &&
                 (static_cast<double>(maxd) >= 16.0 * vol / n ||
                  (pl->directed && mean_span(n, rp, ci) > 16384.0))));
  std::vector<int32_t> rp2, ci2, perm;
  if (pl->sliced) {
    slice_relabel(n, rp, ci, rp2, ci2, perm, pl->slc.slice_off);
    pl->reordered = 1;
  } else if (num_graphs == 1 && o.locality_order != 1 && !pl->directed &&
             (o.locality_order == 2 || n >= (1 << 18))) {
    // Row order: gathers run at L2 speed when neighbouring rows have nearby
    // columns.  Auto relabels by reverse Cuthill-McKee once the vector no longer
    // fits a fraction of one XCD's L2, the caller's entries span more than 2^14
    // labels on average, and the new order shortens that span at least 8x.
    const double span = o.locality_order == 2 ? 0.0 : mean_span(n, rp, ci);
    if (o.locality_order == 2 || span > 16384.0) {
      rcm_order(n, rp, ci, perm);
      relabel_csr(n, rp, ci, perm, rp2, ci2);
      if (o.locality_order == 2 || 8.0 * mean_span(n, rp2.data(), ci2.data()) <= span) {
        pl->reordered = 2;
      } else {
        std::vector<int32_t>().swap(rp2);
        std::vector<int32_t>().swap(ci2);
        std::vector<int32_t>().swap(perm);
      }
    }
  }
  const int32_t* rp1 = pl->reordered ? rp2.data() : rp;   // single-vector labelling
  // candidate work maps: the chosen npt, plus the other sizes when autotuning
  std::vector<int> npts = {pl->npt};
  if (o.autotune && o.nnz_per_thread == 0 && num_graphs == 1 && !pl->sliced)
    for (int c : {8, 16, 32})
      if (c != pl->npt) npts.push_back(c);
  std::vector<std::vector<WorkItem>> item_sets(npts.size());
  std::vector<std::vector<int>> nch_sets(npts.size());
  for (size_t i = 0; i < npts.size(); ++i) build_items(n, rp1, npts[i], item_sets[i], nch_sets[i]);
  std::vector<WorkItem> titems;
  std::vector<int> tnch;
  build_tile_items(n, rp, titems, tnch);
  pl->n_titems = static_cast<int>(titems.size());
  pl->n_tsplit_rows = static_cast<int>(tnch.size());
  pl->tile_w = o.tile_w ? o.tile_w : 64;

  cpaa_status s = CPAA_OK;
  // Host side of the column-sliced layout first (before any device work):
  // packed entry offsets are int, so a pattern whose packed entries (with
  // their run padding) pass kSliceEntryLimit is refused by the sliced layout
  // and keeps row order (the degree-rank labels stay), unless column slices
  // were asked for explicitly.
  HubHost hh;
  std::vector<uint32_t> entries;
  std::vector<WorkItem> sitems;
  std::vector<int> snch;
  if (pl->sliced) {
    int max_slice = 0;
    for (int sl = 0; sl < kSlices; ++sl)
      max_slice = std::max(max_slice, pl->slc.slice_off[sl + 1] - pl->slc.slice_off[sl]);
    // 12 row bits (bigger items) while local columns fit 20 bits below kSliceNone
    pl->slc.row_bits = max_slice <= (1 << 20) - 1 ? kSliceRowBitsMax : 11;
    if (max_slice > (1 << 21) - 2) {
      set_error("column slice too large for the packed entries");
      s = CPAA_EINVAL;
    }
    bool fits = true;
    // the per-item layout (dense partials) serves directed plans and, unless a
    // deterministic plan needs the compact one, the automatic choice
    const int shape = o.slice_shape > 0 ? o.slice_shape : kSliceShapeAuto;
    const bool per_item_layout = pl->directed || shape == kHubConfigs + 1;
    if (s == CPAA_OK && !per_item_layout) {
      hh.cfg = shape - 1;
      fits = build_hub_sliced(n, rp2, ci2, pl->slc.slice_off,
                              o.rows_per_wave > 0 ? o.rows_per_wave : kHubRows, hh);
      std::string why;
      if (fits && !check_hub_map(n, pl->slc.slice_off, hh, why)) {
        set_error("internal error: hub-sliced map check failed (" + why + ")");
        s = CPAA_EINVAL;
      }
    } else if (s == CPAA_OK) {
      fits = build_sliced(n, rp2, ci2, pl->slc.slice_off, pl->slc.row_bits, entries, sitems, snch,
                          pl->slc.item_off);
      for (int sl = 0; sl < kSlices; ++sl)
        pl->slc.max_items =
            std::max(pl->slc.max_items, pl->slc.item_off[sl + 1] - pl->slc.item_off[sl]);
      pl->slc.n_split_rows = static_cast<int>(snch.size());
    }
    if (s == CPAA_OK && !fits) {
      if (o.column_slices == kSlices) {
        set_error("column slices: the packed entries exceed int32 offsets (" +
                  std::to_string(static_cast<long long>(nnz)) + " stored entries)");
        s = CPAA_EINVAL;
      } else {
        pl->sliced = false;
        pl->slc = SlicedMap();
      }
    }
  }
  if (s == CPAA_OK) s = dev_upload(&pl->d_row_ptr, rp, n + 1);
  if (s == CPAA_OK && pl->directed) {
    // out-degree of v = rows that list v, in the single-vector labelling
    const int32_t* ci1 = pl->reordered ? ci2.data() : ci;
    std::vector<int32_t> dout(n, 0);
    for (int64_t j = 0; j < nnz; ++j) ++dout[ci1[j]];
    s = dev_upload(&pl->d_dout, dout.data(), dout.size());
  }
  if (s == CPAA_OK) s = dev_upload(&pl->d_col_idx, ci, static_cast<size_t>(nnz));
  if (s == CPAA_OK && pl->sliced && !hh.items.empty()) {
    HubMap& hm = pl->hub;
    for (int sl = 0; sl <= kSlices; ++sl) {
      hm.item_off[sl] = hh.item_off[sl];
      hm.pofs[sl] = hh.pofs[sl];
    }
    hm.n_long = static_cast<int>(hh.long_out.size());
    hm.n_chunks = static_cast<int>(hh.chunk_long.size());
    int max_items = 0;
    for (int sl = 0; sl < kSlices; ++sl)
      max_items = std::max(max_items, hh.item_off[sl + 1] - hh.item_off[sl]);
    for (int k = 0; k < kHubConfigs; ++k)
      hm.groups[k] = std::max(1, hub_groups_per_slice(k, max_items));
    hm.groups_resid =
        std::max(1, (max_items + kHubResidShape.waves - 1) / kHubResidShape.waves);
    s = dev_upload(&hm.d_entries, hh.entries.data(), hh.entries.size());
    if (s == CPAA_OK) s = dev_upload(&hm.d_items, hh.items.data(), hh.items.size());
    if (s == CPAA_OK) s = dev_upload(&hm.d_mask, hh.mask.data(), hh.mask.size());
    if (s == CPAA_OK) s = dev_upload(&hm.d_base, hh.base.data(), hh.base.size());
    if (s == CPAA_OK) s = dev_upload(&hm.d_chunk_long, hh.chunk_long.data(), hh.chunk_long.size());
    if (s == CPAA_OK) s = dev_upload(&hm.d_long_first, hh.long_first.data(), hh.long_first.size());
    if (s == CPAA_OK) s = dev_upload(&hm.d_long_nch, hh.long_nch.data(), hh.long_nch.size());
    if (s == CPAA_OK) s = dev_upload(&hm.d_long_out, hh.long_out.data(), hh.long_out.size());
    if (s == CPAA_OK) {
      // rounding weights of the residual: sum over the neighbours u of v of (d_u + 3)
      std::vector<double> wr(n);
      parallel_for(n, [&](int64_t v) {
        int64_t w = 0;
        for (int32_t j = rp2[v]; j < rp2[v + 1]; ++j) w += rp2[ci2[j] + 1] - rp2[ci2[j]] + 3;
        wr[v] = static_cast<double>(w);
      });
      s = dev_upload(&hm.d_wround, wr.data(), wr.size());
    }
    hm.cfg = hh.cfg;
    hm.built = s == CPAA_OK;
    std::vector<uint32_t>().swap(hh.entries);
  } else if (s == CPAA_OK && pl->sliced) {
    s = dev_upload(&pl->slc.d_entries, entries.data(), entries.size());
    if (s == CPAA_OK) s = dev_upload(&pl->slc.d_items, sitems.data(), sitems.size());
    if (s == CPAA_OK) s = dev_upload(&pl->slc.d_split_nchunks, snch.data(), snch.size());
  }
  if (pl->n_drop > 0) {
    // single-vector labels -> the caller's: through the relabelling, then the
    // vertices that were kept
    if (pl->reordered)
      for (int32_t& v : perm) v = keep[v];
    else
      perm = keep;
    if (s == CPAA_OK) s = dev_upload(&pl->d_dropped, dropped.data(), dropped.size());
  }
  if (pl->reordered) {
    if (s == CPAA_OK) s = dev_upload(&pl->d_rp_w1, rp2.data(), rp2.size());
    if (s == CPAA_OK) s = dev_upload(&pl->d_ci_w1, ci2.data(), ci2.size());
  } else {
    pl->d_rp_w1 = pl->d_row_ptr;
    pl->d_ci_w1 = pl->d_col_idx;
  }
  if (pl->reordered || pl->n_drop > 0)
    if (s == CPAA_OK) s = dev_upload(&pl->d_perm, perm.data(), perm.size());
  pl->maps.resize(npts.size());
  for (size_t i = 0; i < npts.size() && s == CPAA_OK; ++i) {
    WorkMap& m = pl->maps[i];
    m.npt = npts[i];
    m.n_items = static_cast<int>(item_sets[i].size());
    m.n_split_rows = static_cast<int>(nch_sets[i].size());
    pl->max_split_rows = std::max(pl->max_split_rows, m.n_split_rows);
    s = dev_upload(&m.d_items, item_sets[i].data(), item_sets[i].size());
    if (s == CPAA_OK) s = dev_upload(&m.d_split_nchunks, nch_sets[i].data(), nch_sets[i].size());
  }
  if (s == CPAA_OK) select_map(pl, 0);
  if (s == CPAA_OK) s = dev_upload(&pl->d_titems, titems.data(), titems.size());
  if (s == CPAA_OK) s = dev_upload(&pl->d_tsplit_nchunks, tnch.data(), tnch.size());
  if (s == CPAA_OK && num_graphs > 1) {
    pl->h_graph_ptr.assign(gp, gp + num_graphs + 1);
    std::vector<int64_t>& gnnz = pl->h_graph_nnz;
    gnnz.assign(num_graphs, 0);
    for (int gi = 0; gi < num_graphs; ++gi) {
      gnnz[gi] = static_cast<int64_t>(rp[gp[gi + 1]]) - rp[gp[gi]];
      pl->max_graph_n = std::max(pl->max_graph_n, gp[gi + 1] - gp[gi]);
      pl->max_graph_nnz = std::max(pl->max_graph_nnz, gnnz[gi]);
    }
    // size classes: class 0 holds graphs with more than max_n/2 vertices, class 1
    // more than max_n/4, class 2 more than max_n/8, class 3 the rest; each class
    // is launched with the LDS its own largest graph needs (and its own
    // workgroup size), so small graphs get more workgroups per CU
    auto cls = [&](int gi) {
      const int ng = gp[gi + 1] - gp[gi];
      return ng * 2 > pl->max_graph_n ? 0
             : ng * 4 > pl->max_graph_n ? 1
             : ng * 8 > pl->max_graph_n ? 2
                                        : 3;
    };
    std::vector<int32_t> order(num_graphs);
    for (int gi = 0; gi < num_graphs; ++gi) order[gi] = gi;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      return cls(a) != cls(b) ? cls(a) < cls(b) : gnnz[a] > gnnz[b];
    });
    for (int k = 0; k <= kGraphClasses; ++k) pl->graph_cls_off[k] = 0;
    for (int gi = 0; gi < num_graphs; ++gi) {
      const int k = cls(gi);
      ++pl->graph_cls_off[k + 1];
      pl->graph_cls_n[k] = std::max(pl->graph_cls_n[k], gp[gi + 1] - gp[gi]);
    }
    for (int k = 0; k < kGraphClasses; ++k) pl->graph_cls_off[k + 1] += pl->graph_cls_off[k];
    s = dev_upload(&pl->d_graph_ptr, gp, num_graphs + 1);
    if (s == CPAA_OK) s = dev_upload(&pl->d_graph_order, order.data(), order.size());
    if (s == CPAA_OK) s = dev_alloc(&pl->d_queue, kGraphClasses);
    if (s == CPAA_OK) s = build_graph_state(pl, rp, ci, gp);
  }
  if (s == CPAA_OK) {
    if (hipEventCreate(&pl->ev_begin) != hipSuccess || hipEventCreate(&pl->ev_end) != hipSuccess ||
        hipEventCreateWithFlags(&pl->ev_poll[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&pl->ev_poll[1], hipEventDisableTiming) != hipSuccess) {
      set_error("hipEventCreate failed");
      s = CPAA_EDEVICE;
    }
  }
  if (s != CPAA_OK) {
    cpaa_plan_destroy(pl);
    return s;
  }
  *out = pl;
  return CPAA_OK;
}

cpaa_status cpaa_plan_info_get(cpaa_plan_t pl, cpaa_plan_info* info) {
  if (!pl || !info) {
    set_error("cpaa_plan_info_get: null argument");
    return CPAA_EINVAL;
  }
  std::memset(info, 0, sizeof(*info));
  info->n = pl->n_caller;
  info->nnz = pl->nnz;
  info->num_graphs = pl->num_graphs;
  info->reordered = pl->reordered;
  info->max_degree = pl->max_deg;
  info->split_rows = pl->n_split_rows;
  info->nnz_per_thread = pl->npt;
  info->work_items = pl->n_items;
  info->tile_w = pl->tile_w;
  info->c = pl->c;
  info->beta = pl->beta;
  info->vol = pl->vol;
  info->k_cap_global = mass_rule_terms(pl, 1e-6);
  info->column_slices = pl->sliced ? kSlices : 1;
  info->spectrum_lo = pl->lam_lo;
  info->directed = pl->directed ? 1 : 0;
  info->slice_shape = pl->hub.built ? pl->hub.cfg + 1 : (pl->sliced ? kHubConfigs + 1 : 0);
  info->slice_partials = pl->hub.built ? pl->hub.pofs[kSlices] : 0;
  return CPAA_OK;
}

}  // extern "C"
