// Host setup: ILUT(tau, m) of the stiffness matrix (Section 3, "Smoother").
//
// Dual-threshold incomplete LU, row by row (i-k-j order), pivots k < i taken
// in increasing order:
//   rule 1  an entry is dropped when its magnitude is below
//           tau_i = tau * (sum_j |a_ij|) / nnz_i, the average magnitude of the
//           stored entries of the original row; applied to each multiplier
//           w_k / u_kk before it is used, and to the final row (never to the
//           diagonal);
//   rule 2  only the M largest entries are kept, M = floor(m nnz(A) / n),
//           either per part (M in the strict lower part and M in the strict
//           upper part), per row (M off-diagonal entries in total) or half
//           per part (floor(M/2) in each part); magnitudes are ranked in
//           single precision and ties go to the smaller column; exact zeros
//           are never stored.
// A zero or non-finite pivot fails the factorisation (no substitution).
//
// Rows depend on earlier rows only through the pivots they meet, and each
// row's final pivot is usually its left neighbour; the factorisation is
// therefore pipelined over threads: thread t takes rows t, t+T, ..., and a
// row waits for a pivot row only when it reaches it.  Every row is computed
// with exactly the operations of the sequential algorithm, so the result
// does not depend on the thread count.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <functional>
#include <memory>
#include <thread>

#include "pmg_host.hpp"

namespace pmg {

namespace {

struct Entry {
  int32_t j;
  double v;
};

// Append-only storage whose blocks never move, so rows published by one
// thread stay valid while others read them.
struct Arena {
  static constexpr size_t kBlock = size_t(1) << 20;
  std::vector<std::unique_ptr<Entry[]>> blocks;
  size_t used = kBlock;
  Entry* alloc(size_t n) {
    if (n > kBlock) {
      blocks.emplace_back(new Entry[n]);
      used = kBlock;
      return blocks.back().get();
    }
    if (used + n > kBlock) {
      blocks.emplace_back(new Entry[kBlock]);
      used = 0;
    }
    Entry* p = blocks.back().get() + used;
    used += n;
    return p;
  }
};

struct RowRef {
  const Entry* L = nullptr;  // strict lower, sorted by column
  const Entry* U = nullptr;  // diagonal first, then strict upper sorted
  int32_t nl = 0, nu = 0;    // nu includes the diagonal
};

// Magnitudes are ranked in single precision: entries equal in exact
// arithmetic (mirror images on a symmetric grid) then tie and are ordered by
// column, not by the last bits of their FP64 rounding.
bool mag_before(const Entry& a, const Entry& b) {
  float x = (float)std::fabs(a.v), y = (float)std::fabs(b.v);
  if (x != y) return x > y;
  return a.j < b.j;
}

bool col_before(const Entry& a, const Entry& b) { return a.j < b.j; }

}  // namespace

int ilut_factor(const Csr& A, double tau, double fill, int mode, int threads, Csr& Lout, Csr& Uout,
                int& bad_row) {
  const int n = A.nrows;
  const int64_t nnzA = A.nnz();
  const int64_t M = fill > 0 ? (int64_t)std::floor(fill * (double)nnzA / (double)n) : (int64_t)n;
  threads = std::max(1, std::min(threads, 64));
  std::vector<RowRef> rows(n);
  std::unique_ptr<std::atomic<int>[]> done(new std::atomic<int>[n]);
  for (int i = 0; i < n; ++i) done[i].store(0, std::memory_order_relaxed);
  std::atomic<int> failed_row(-1);
  std::vector<Arena> arenas(threads);

  auto worker = [&](int t) {
    std::vector<double> w(n, 0.0);
    std::vector<char> used(n, 0);
    std::vector<int32_t> touched;
    std::vector<int32_t> heap;  // min-heap of touched columns < i
    std::vector<Entry> lo, up;
    touched.reserve(4096);
    Arena& arena = arenas[t];
    for (int i = t; i < n; i += threads) {
      {
        int fr = failed_row.load(std::memory_order_relaxed);
        if (fr >= 0 && fr < i) break;
      }
      touched.clear();
      heap.clear();
      double rs = 0.0;
      for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        int32_t j = A.ci[k];
        w[j] = A.v[k];
        if (!used[j]) {
          used[j] = 1;
          touched.push_back(j);
          if (j < i) heap.push_back(j);
        }
        rs += std::fabs(A.v[k]);
      }
      std::make_heap(heap.begin(), heap.end(), std::greater<int32_t>());
      const int64_t nzi = A.rp[i + 1] - A.rp[i];
      const double taui = nzi > 0 ? tau * (rs / (double)nzi) : 0.0;
      bool fail = false;
      while (!heap.empty()) {
        std::pop_heap(heap.begin(), heap.end(), std::greater<int32_t>());
        int32_t k = heap.back();
        heap.pop_back();
        if (w[k] == 0.0) continue;
        // wait for row k
        while (!done[k].load(std::memory_order_acquire)) {
          int fr = failed_row.load(std::memory_order_relaxed);
          if (fr >= 0 && fr <= k) {  // row k can no longer complete
            fail = true;
            break;
          }
          std::this_thread::yield();
        }
        if (fail) break;
        const RowRef& rk = rows[k];
        double ukk = rk.U[0].v;
        double lk = w[k] / ukk;
        if (std::fabs(lk) < taui) {
          w[k] = 0.0;
          continue;
        }
        w[k] = lk;
        for (int32_t s = 1; s < rk.nu; ++s) {
          int32_t j = rk.U[s].j;
          if (!used[j]) {
            used[j] = 1;
            touched.push_back(j);
            w[j] = 0.0;
            if (j < i) {
              heap.push_back(j);
              std::push_heap(heap.begin(), heap.end(), std::greater<int32_t>());
            }
          }
          w[j] -= lk * rk.U[s].v;
        }
      }
      double d = used[i] ? w[i] : 0.0;
      if (!fail && (!(d != 0.0) || !std::isfinite(d))) {
        int cur = failed_row.load();
        while ((cur < 0 || cur > i) && !failed_row.compare_exchange_weak(cur, i)) {
        }
        fail = true;
      }
      if (!fail) {
        lo.clear();
        up.clear();
        for (int32_t j : touched) {
          if (j == i) continue;
          double x = w[j];
          if (x == 0.0 || std::fabs(x) < taui) continue;
          (j < i ? lo : up).push_back({j, x});
        }
        if (mode != 1) {
          const int64_t Mp = mode == 2 && fill > 0 ? M / 2 : M;  // fill <= 0: no limit in any mode
          if ((int64_t)lo.size() > Mp) {
            std::nth_element(lo.begin(), lo.begin() + Mp, lo.end(), mag_before);
            lo.resize(Mp);
          }
          if ((int64_t)up.size() > Mp) {
            std::nth_element(up.begin(), up.begin() + Mp, up.end(), mag_before);
            up.resize(Mp);
          }
        } else {
          std::vector<Entry> all(lo);
          all.insert(all.end(), up.begin(), up.end());
          if ((int64_t)all.size() > M) {
            std::nth_element(all.begin(), all.begin() + M, all.end(), mag_before);
            all.resize(M);
          }
          lo.clear();
          up.clear();
          for (auto& e : all) (e.j < i ? lo : up).push_back(e);
        }
        std::sort(lo.begin(), lo.end(), col_before);
        std::sort(up.begin(), up.end(), col_before);
        Entry* Lp = arena.alloc(lo.size() ? lo.size() : 1);
        std::copy(lo.begin(), lo.end(), Lp);
        Entry* Up = arena.alloc(up.size() + 1);
        Up[0] = {i, d};
        std::copy(up.begin(), up.end(), Up + 1);
        rows[i].L = Lp;
        rows[i].U = Up;
        rows[i].nl = (int32_t)lo.size();
        rows[i].nu = (int32_t)up.size() + 1;
      }
      for (int32_t j : touched) {
        used[j] = 0;
        w[j] = 0.0;
      }
      if (fail) break;
      done[i].store(1, std::memory_order_release);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < threads; ++t) pool.emplace_back(worker, t);
  worker(0);
  for (auto& th : pool) th.join();
  if (failed_row.load() >= 0) {
    bad_row = failed_row.load();
    return 4;  // PMG_EZEROPIVOT
  }
  Lout = Csr();
  Uout = Csr();
  Lout.nrows = Lout.ncols = Uout.nrows = Uout.ncols = n;
  Lout.rp.assign((size_t)n + 1, 0);
  Uout.rp.assign((size_t)n + 1, 0);
  for (int i = 0; i < n; ++i) {
    Lout.rp[i + 1] = Lout.rp[i] + rows[i].nl;
    Uout.rp[i + 1] = Uout.rp[i] + rows[i].nu;
  }
  Lout.ci.resize(Lout.rp[n]);
  Lout.v.resize(Lout.rp[n]);
  Uout.ci.resize(Uout.rp[n]);
  Uout.v.resize(Uout.rp[n]);
  for (int i = 0; i < n; ++i) {
    for (int s = 0; s < rows[i].nl; ++s) {
      Lout.ci[Lout.rp[i] + s] = rows[i].L[s].j;
      Lout.v[Lout.rp[i] + s] = rows[i].L[s].v;
    }
    for (int s = 0; s < rows[i].nu; ++s) {
      Uout.ci[Uout.rp[i] + s] = rows[i].U[s].j;
      Uout.v[Uout.rp[i] + s] = rows[i].U[s].v;
    }
  }
  return 0;
}

// ----------------------------------------------------------------- ordering
// Lines along x are indexed by their (y[, z]) position.  Boxes of lines are
// split across the longest side by a separator p lines wide; the emitted
// order is first part, second part, separator.  An explicit stack replays
// that order: a box to split pushes (separator, second, first) so that the
// first part is processed next.
std::vector<int32_t> line_ordering(int dim, int nint, int p, int ordering, int leaf) {
  const int64_t nlines = dim == 2 ? nint : (int64_t)nint * nint;
  std::vector<int32_t> lines;
  lines.reserve(nlines);
  if (ordering == 0) {
    for (int64_t l = 0; l < nlines; ++l) lines.push_back((int32_t)l);
  } else {
    struct Box {
      int y0, y1, z0, z1;
      bool whole;  // emit without cutting (a separator)
    };
    std::vector<Box> stack;
    stack.push_back({0, nint, 0, dim == 2 ? 1 : nint, false});
    while (!stack.empty()) {
      Box b = stack.back();
      stack.pop_back();
      const int ey = b.y1 - b.y0, ez = b.z1 - b.z0;
      if (ey <= 0 || ez <= 0) continue;
      const int longest = std::max(ey, ez);
      if (b.whole || ey * ez <= leaf || longest < 2 * p + 3) {
        for (int z = b.z0; z < b.z1; ++z)
          for (int y = b.y0; y < b.y1; ++y) lines.push_back(y + nint * z);
        continue;
      }
      if (ey >= ez) {
        const int m = b.y0 + (ey - p) / 2;
        stack.push_back({m, m + p, b.z0, b.z1, true});
        stack.push_back({m + p, b.y1, b.z0, b.z1, false});
        stack.push_back({b.y0, m, b.z0, b.z1, false});
      } else {
        const int m = b.z0 + (ez - p) / 2;
        stack.push_back({b.y0, b.y1, m, m + p, true});
        stack.push_back({b.y0, b.y1, m + p, b.z1, false});
        stack.push_back({b.y0, b.y1, b.z0, m, false});
      }
    }
  }
  std::vector<int32_t> perm((size_t)nlines * nint);
  size_t i = 0;
  for (int32_t l : lines)
    for (int x = 0; x < nint; ++x) perm[i++] = l * nint + x;
  return perm;
}

namespace {

struct NdBlock {
  int64_t l0, l1;  // positions of its lines in the ordering, [l0, l1)
  int height;      // 0 for an uncut box, 1 + the children's for a separator
};

// The blocks of the nested-dissection order, in emission order, following
// the same cuts as line_ordering.  Returns the box's height (-1 if empty).
int nd_blocks(int y0, int y1, int z0, int z1, bool whole, int nint, int p, int leaf, int64_t& pos,
              std::vector<NdBlock>& out) {
  const int ey = y1 - y0, ez = z1 - z0;
  if (ey <= 0 || ez <= 0) return -1;
  const int longest = std::max(ey, ez);
  if (whole || ey * ez <= leaf || longest < 2 * p + 3) {
    out.push_back({pos, pos + (int64_t)ey * ez, 0});
    pos += (int64_t)ey * ez;
    return 0;
  }
  int h1, h2;
  NdBlock sep;
  if (ey >= ez) {
    const int m = y0 + (ey - p) / 2;
    h1 = nd_blocks(y0, m, z0, z1, false, nint, p, leaf, pos, out);
    h2 = nd_blocks(m + p, y1, z0, z1, false, nint, p, leaf, pos, out);
    sep = {pos, pos + (int64_t)p * ez, 0};
  } else {
    const int m = z0 + (ez - p) / 2;
    h1 = nd_blocks(y0, y1, z0, m, false, nint, p, leaf, pos, out);
    h2 = nd_blocks(y0, y1, m + p, z1, false, nint, p, leaf, pos, out);
    sep = {pos, pos + (int64_t)ey * p, 0};
  }
  sep.height = std::max(std::max(h1, h2), -1) + 1;
  pos = sep.l1;
  out.push_back(sep);
  return sep.height;
}

}  // namespace

std::vector<int32_t> factor_ticket_order(int dim, int nint, int p, int ordering, int leaf) {
  const int64_t nlines = dim == 2 ? nint : (int64_t)nint * nint;
  std::vector<NdBlock> blocks;
  if (ordering == 0) {
    blocks.push_back({0, nlines, 0});
  } else {
    int64_t pos = 0;
    nd_blocks(0, nint, 0, dim == 2 ? 1 : nint, false, nint, p, leaf, pos, blocks);
  }
  int hmax = 0;
  for (const NdBlock& b : blocks) hmax = std::max(hmax, b.height);
  std::vector<int32_t> order;
  order.reserve((size_t)nlines * nint);
  for (int h = 0; h <= hmax; ++h) {
    std::vector<const NdBlock*> lev;
    int64_t longest = 0;
    for (const NdBlock& b : blocks)
      if (b.height == h) {
        lev.push_back(&b);
        longest = std::max(longest, (b.l1 - b.l0) * nint);
      }
    for (int64_t r = 0; r < longest; ++r)
      for (const NdBlock* b : lev)
        if (r < (b->l1 - b->l0) * nint) order.push_back((int32_t)(b->l0 * nint + r));
  }
  return order;
}

std::vector<int32_t> line_segments(int dim, int nint, int p, int ordering, int leaf, int max_rows) {
  const int64_t nlines = dim == 2 ? nint : (int64_t)nint * nint;
  std::vector<NdBlock> blocks;
  if (ordering == 0) {
    blocks.push_back({0, nlines, 0});
  } else {
    int64_t pos = 0;
    nd_blocks(0, nint, 0, dim == 2 ? 1 : nint, false, nint, p, leaf, pos, blocks);
  }
  const int64_t k = std::max<int64_t>(1, max_rows / nint);  // lines per segment
  std::vector<int32_t> starts;
  for (const NdBlock& b : blocks)
    for (int64_t l = b.l0; l < b.l1; l += k) starts.push_back((int32_t)(l * nint));
  starts.push_back((int32_t)(nlines * nint));
  return starts;
}

Csr permute(const Csr& A, const std::vector<int32_t>& perm, int threads) {
  const int n = A.nrows;
  std::vector<int32_t> inv(n);
  for (int i = 0; i < n; ++i) inv[perm[i]] = i;
  Csr B;
  B.nrows = B.ncols = n;
  B.rp.assign((size_t)n + 1, 0);
  for (int i = 0; i < n; ++i) B.rp[i + 1] = B.rp[i] + (A.rp[perm[i] + 1] - A.rp[perm[i]]);
  B.ci.resize(B.rp[n]);
  B.v.resize(B.rp[n]);
  auto work = [&](int lo, int hi) {
    std::vector<Entry> tmp;
    for (int i = lo; i < hi; ++i) {
      const int r = perm[i];
      tmp.clear();
      for (int64_t k = A.rp[r]; k < A.rp[r + 1]; ++k) tmp.push_back({inv[A.ci[k]], A.v[k]});
      std::sort(tmp.begin(), tmp.end(), col_before);
      int64_t o = B.rp[i];
      for (const Entry& e : tmp) {
        B.ci[o] = e.j;
        B.v[o] = e.v;
        ++o;
      }
    }
  };
  threads = std::max(1, threads);
  std::vector<std::thread> pool;
  const int chunk = (n + threads - 1) / threads;
  for (int t = 0; t < threads; ++t) {
    const int lo = t * chunk, hi = std::min(n, lo + chunk);
    if (lo < hi) pool.emplace_back(work, lo, hi);
  }
  for (auto& th : pool) th.join();
  return B;
}

}  // namespace pmg
