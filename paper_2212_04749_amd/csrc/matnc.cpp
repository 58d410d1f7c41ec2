// libmatnc: plan construction, binding, execution and the C ABI.
//
// Method (main text "Multiple-amplitude simulation with static and optimal
// tensor reuse"; Supplementary Secs. III-IV): the k networks of a bitstring
// batch share every tensor computed before the first output index is met.
// For a node v of the contraction tree, all bitstrings with the same
// projection onto the closed outputs below v share v's tensor, so v is
// computed once per distinct projection (w(v) instances) -- the optimal
// reuse whose cost is Eq. (1).  Instances are computed breadth-first per
// tree level in batched launches, each reading its operands through gather
// maps.  Slicing (Sec. IV.B) fixes the sliced indices per slice; nodes with
// no sliced index below them are computed once and kept (stem cache), the
// others once per slice, and the root instances of every slice are added in
// FP64 into the caller's amplitudes in slice order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <exception>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/matnc.h"
#include "desc.h"
#include "kernels.h"
#include "plan.h"

using namespace matnc;

struct matnc_network_s {
  Network net;
};
struct matnc_plan_s {
  Plan p;
};
struct matnc_queue_s {
  std::vector<matnc_plan> plans;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> key;  // amplitude buffers, XEB slot and plan generations of the captured graph
};

namespace {

thread_local std::string g_err;

struct Err : std::runtime_error {
  int code;
  Err(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(int code, const std::string& msg) { throw Err(code, msg); }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(MATNC_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class F>
int guarded(F&& f) {
  try {
    f();
    return MATNC_OK;
  } catch (const Err& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host memory exhausted";
    return MATNC_E_INVALID;
  } catch (const std::exception& e) {
    g_err = e.what();
    return MATNC_E_INVALID;
  } catch (...) {
    g_err = "unknown error";
    return MATNC_E_INVALID;
  }
}

constexpr uint64_t kAlign = 256;

// Complex-half plans: how many intermediates may be stored in FP16 unless
// the caller sets matnc_plan_options_t.half_nodes.  With N such tensors the
// amplitudes carry relative errors of rms e ~ 2.8e-4 sqrt(N); the linear XEB
// of K amplitudes then moves by about 2 e / sqrt(K) (independent errors,
// Porter-Thomas amplitudes).  Keeping three times that within the 1e-4 XEB
// bar gives N <= K / kAmpsPerHalfNode.  The errors are not independent in
// general (which tensors are rounded matters): on the 6x6 depth-14 workload
// the XEB of 16 384 amplitudes stays within 4.5e-5 of complex64's up to 24
// FP16 tensors and jumps to 1.5e-4 at 28, while the pass gets only 2%
// faster above 12; kMaxHalfNodes = 16 keeps that margin and e near 1e-3.
constexpr int64_t kAmpsPerHalfNode = 282;
constexpr int kMaxHalfNodes = 16;

// bytes per stored element of node v: complex64 (8) unless the plan is
// complex-half and v is an FP16-stored branch tensor (4)
inline uint64_t eb_of(const Plan& P, int v) { return P.nodes[v].half_store ? 4 : 8; }

uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// ---------------------------------------------------------------------------
// plan construction

void build_structure(Plan& P) {
  const Network& N = P.net;
  const int nt = N.n_tensors;
  P.n_nodes = 2 * nt - 1;
  P.nodes.assign(P.n_nodes, PNode());

  std::unordered_map<int, int> out_qubit;  // output index -> qubit
  for (int q = 0; q < N.n_qubits; ++q) out_qubit[N.out_index[q]] = q;
  std::vector<char> is_open(N.n_qubits, 0);
  for (int q : P.open_qubits) is_open[q] = 1;
  std::unordered_map<int, int> slice_bit;
  for (size_t j = 0; j < P.sliced.size(); ++j) slice_bit[P.sliced[j]] = (int)j;

  // free index sets (unordered for now)
  std::vector<std::vector<int>> freeset(P.n_nodes);
  for (int t = 0; t < nt; ++t) {
    PNode& L = P.nodes[t];
    std::vector<std::pair<int, int>> sl;
    for (int i : N.idx[t]) {
      auto oq = out_qubit.find(i);
      if (oq != out_qubit.end() && !is_open[oq->second]) {
        L.omask |= 1ull << oq->second;
        continue;
      }
      auto sb = slice_bit.find(i);
      if (sb != slice_bit.end()) {
        sl.push_back({sb->second, i});
        continue;
      }
      freeset[t].push_back(i);
    }
    std::sort(sl.begin(), sl.end());
    for (auto& x : sl) {
      L.sl_bits.push_back(x.first);
      L.sl_index.push_back(x.second);
    }
    if ((int)L.sl_bits.size() > kMaxLeafSliced) fail(MATNC_E_INVALID, "a tensor holds more than 16 sliced indices");
    L.dep = !L.sl_bits.empty();
  }
  // internal nodes; death time of contracted indices
  std::unordered_map<int, int> death;
  for (int j = 0; j < nt - 1; ++j) {
    const int v = nt + j;
    const int a = P.pairs[j].first, b = P.pairs[j].second;
    PNode& V = P.nodes[v];
    V.a = a;
    V.b = b;
    P.nodes[a].parent = v;
    P.nodes[b].parent = v;
    V.omask = P.nodes[a].omask | P.nodes[b].omask;
    V.dep = P.nodes[a].dep || P.nodes[b].dep;
    std::vector<int> fa = freeset[a], fb = freeset[b];
    std::sort(fa.begin(), fa.end());
    std::sort(fb.begin(), fb.end());
    std::vector<int> shared, out;
    std::set_intersection(fa.begin(), fa.end(), fb.begin(), fb.end(), std::back_inserter(shared));
    std::set_symmetric_difference(fa.begin(), fa.end(), fb.begin(), fb.end(), std::back_inserter(out));
    for (int i : shared) death[i] = v;
    freeset[v] = out;
  }
  // storage order: latest death lowest; open outputs (never contracted)
  // first, in ascending qubit order
  auto key_of = [&](int i) {
    auto oq = out_qubit.find(i);
    if (oq != out_qubit.end()) return std::make_pair(-1LL, (long long)oq->second);
    auto d = death.find(i);
    const long long dt = d == death.end() ? (long long)INT_MAX : (long long)d->second;
    return std::make_pair(-dt, (long long)i);
  };
  P.max_rank = 0;
  for (int v = 0; v < P.n_nodes; ++v) {
    std::vector<int> f = freeset[v];
    std::sort(f.begin(), f.end(), [&](int x, int y) { return key_of(x) < key_of(y); });
    P.nodes[v].idx = f;
    P.max_rank = std::max<int>(P.max_rank, (int)f.size());
  }
  if (P.max_rank > P.max_rank_cap)
    fail(MATNC_E_RANK, "largest tensor has rank " + std::to_string(P.max_rank) + " > max_rank " +
                           std::to_string(P.max_rank_cap));
  if (P.max_rank > 32) fail(MATNC_E_RANK, "ranks above 32 are not supported");
}

void build_reuse(Plan& P) {
  const int nt = P.net.n_tensors;
  // distinct projections per node
  std::map<uint64_t, std::vector<uint64_t>> cache;
  for (int v = 0; v < P.n_nodes; ++v) {
    const uint64_t m = P.nodes[v].omask;
    auto it = cache.find(m);
    if (it == cache.end()) {
      std::vector<uint64_t> ks;
      ks.reserve(P.words.size());
      for (uint64_t w : P.words) ks.push_back(w & m);
      std::sort(ks.begin(), ks.end());
      ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
      it = cache.emplace(m, std::move(ks)).first;
    }
    P.nodes[v].keys = it->second;
  }
  auto find = [](const std::vector<uint64_t>& ks, uint64_t u) -> int32_t {
    auto it = std::lower_bound(ks.begin(), ks.end(), u);
    return (int32_t)(it - ks.begin());
  };
  for (int v = nt; v < P.n_nodes; ++v) {
    PNode& V = P.nodes[v];
    const PNode& A = P.nodes[V.a];
    const PNode& B = P.nodes[V.b];
    V.ga.resize(V.keys.size());
    V.gb.resize(V.keys.size());
    for (size_t j = 0; j < V.keys.size(); ++j) {
      V.ga[j] = find(A.keys, V.keys[j] & A.omask);
      V.gb[j] = find(B.keys, V.keys[j] & B.omask);
    }
  }
  const PNode& R = P.nodes[P.n_nodes - 1];
  P.n_unique = (int64_t)P.nodes[P.n_nodes - 1].keys.size();
  {
    std::vector<uint64_t> u = P.words;
    std::sort(u.begin(), u.end());
    P.n_unique = (int64_t)(std::unique(u.begin(), u.end()) - u.begin());
  }
}

// fan table: the output instances j grouped by the A instance they read
// (ga[j]), each group cut into rows of `slots` entries (-1 = empty slot)
void make_fan(const std::vector<int32_t>& ga, int slots, std::vector<int32_t>& out, int64_t& n_fan) {
  std::vector<int32_t> order(ga.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return ga[x] < ga[y]; });
  out.clear();
  n_fan = 0;
  size_t i = 0;
  while (i < order.size()) {
    size_t e = i;
    while (e < order.size() && ga[order[e]] == ga[order[i]]) ++e;
    for (size_t c = i; c < e; c += (size_t)slots) {
      for (int t = 0; t < slots; ++t) out.push_back(c + t < e ? order[c + t] : -1);
      ++n_fan;
    }
    i = e;
  }
}

// tile-order block (NodeDesc::fan_rows) of units whose A instances are
// a_of(0 .. n-1) (adjacent units with equal values share one): when the A
// instance is too large for the caches to keep it between blocks of `dflt`
// units (64 MiB), the median number of units per A instance if that is 4 or
// more (a block then reads about one or two A instances per tile), else dflt
template <typename F>
int32_t block_units(size_t n, F a_of, uint64_t a_inst_bytes, int32_t dflt) {
  if (n == 0 || a_inst_bytes < (64ull << 20)) return dflt;
  std::vector<int64_t> runs;
  int64_t run = 0;
  for (size_t r = 0; r < n; ++r) {
    ++run;
    if (r + 1 == n || a_of(r + 1) != a_of(r)) {
      runs.push_back(run);
      run = 0;
    }
  }
  std::nth_element(runs.begin(), runs.begin() + runs.size() / 2, runs.end());
  const int64_t g = runs[runs.size() / 2];
  return g >= 4 ? (int32_t)g : dflt;
}

// ... of a fan table (rows of `slots` output instances)
int32_t fan_block_rows(const std::vector<int32_t>& fanv, int slots, const std::vector<int32_t>& ga,
                       uint64_t a_inst_bytes) {
  return block_units(fanv.size() / (size_t)slots, [&](size_t r) { return ga[fanv[r * slots]]; }, a_inst_bytes, 2);
}

// ... of the instances of a plain step
int32_t plain_block_units(const std::vector<int32_t>& ga, uint64_t a_inst_bytes) {
  return block_units(ga.size(), [&](size_t j) { return ga[j]; }, a_inst_bytes, 1);
}

void build_steps(Plan& P) {
  const int nt = P.net.n_tensors;
  P.n_mfma = 0;
  P.cmac_single = P.cmac_multi = P.cmac_inv = P.cmac_total = 0;
  P.bytes_slice = P.bytes_inv = 0;
  const double nsl = std::ldexp(1.0, (int)P.sliced.size());
  // complex-half storage policy: the P.half_nodes intermediates whose steps
  // carry the most estimated FP32 time are stored in FP16 with per-instance
  // exponents (they then run on the FP16 MFMA kernels and move half the
  // bytes); leaves and the other intermediates stay FP32.  Each FP16 tensor
  // adds one rounding of relative rms about 2^-11 / sqrt(3) = 2.8e-4, so
  // their number is the precision budget of the plan (see kMaxHalfNodes).
  std::vector<double> t32(P.n_nodes, 0.0);
  for (int v = nt; v < P.n_nodes; ++v) {
    const PNode& V = P.nodes[v];
    const PNode& ca = P.nodes[V.a];
    const PNode& cb = P.nodes[V.b];
    std::vector<int> fa(ca.idx), fb(cb.idx);
    std::sort(fa.begin(), fa.end());
    std::sort(fb.begin(), fb.end());
    std::vector<int> sh;
    std::set_intersection(fa.begin(), fa.end(), fb.begin(), fb.end(), std::back_inserter(sh));
    const int kb = (int)sh.size();
    const int ra = (int)std::max(fa.size(), fb.size()), rb = (int)std::min(fa.size(), fb.size());
    const int mb = ra - kb, nb = rb - kb;
    const double w = (double)V.keys.size();
    const double wa = (double)(fa.size() >= fb.size() ? ca : cb).keys.size();
    const double wb = (double)(fa.size() >= fb.size() ? cb : ca).keys.size();
    const double flops = 8.0 * w * std::ldexp(1.0, mb + nb + kb);
    const double bytes = 8.0 * (w * std::ldexp(1.0, (int)V.idx.size()) + wa * std::ldexp(1.0, ra) +
                                wb * std::ldexp(1.0, rb));
    const bool gemm = nb + kb >= 8 && mb >= 6 && nb >= 5 && kb >= 3;
    t32[v] = std::max(flops / (gemm ? 100e12 : 40e12), bytes / 3e12) * (V.dep ? nsl : 1.0);
  }
  std::vector<char> half(P.n_nodes, 0);
  if (P.precision == MATNC_CHALF && P.half_nodes > 0) {
    std::vector<int> order;
    for (int v = nt; v < P.n_nodes; ++v) order.push_back(v);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return t32[x] > t32[y]; });
    for (size_t i = 0; i < order.size() && (int)i < P.half_nodes; ++i) half[order[i]] = 1;
  }
  P.n_half = 0;
  for (int v = 0; v < P.n_nodes; ++v) {
    P.nodes[v].half_store = half[v] != 0;
    P.n_half += half[v] ? 1 : 0;
  }
  for (int v = nt; v < P.n_nodes; ++v) {
    PNode& V = P.nodes[v];
    const bool hm = V.half_store;  // FP16 output: FP16-product MFMA kernels
    const PNode& ca = P.nodes[V.a];
    const PNode& cb = P.nodes[V.b];
    V.swap = cb.idx.size() > ca.idx.size();
    const PNode& A = V.swap ? cb : ca;
    const PNode& B = V.swap ? ca : cb;
    if (V.swap) std::swap(V.ga, V.gb);
    std::vector<int> sa(A.idx), sb(B.idx);
    std::vector<int> sa_sorted(sa), sb_sorted(sb);
    std::sort(sa_sorted.begin(), sa_sorted.end());
    std::sort(sb_sorted.begin(), sb_sorted.end());
    V.M.clear();
    V.N.clear();
    V.K.clear();
    for (int i : A.idx) {
      if (std::binary_search(sb_sorted.begin(), sb_sorted.end(), i))
        V.K.push_back(i);
      else
        V.M.push_back(i);
    }
    for (int i : B.idx)
      if (!std::binary_search(sa_sorted.begin(), sa_sorted.end(), i)) V.N.push_back(i);
    const int mb = (int)V.M.size(), nb = (int)V.N.size(), kb = (int)V.K.size();
    V.kernel = 0;
    V.cfg = -1;
    if (nb + kb >= 8) {
      // MFMA tiles: prefer the widest N tile that fits
      if (!hm) {
        const int order[] = {1, 0, 3, 2};
        for (int c : order) {
          if (mfma_config_fits(c, mb, nb, kb)) {
            V.kernel = 1;
            V.cfg = c;
            break;
          }
        }
      } else {
        const int order[] = {0, 1, 3, 2, 4};
        for (int c : order) {
          if (mfma_h_config_fits(c, mb, nb, kb)) {
            V.kernel = 1;
            V.cfg = c;
            break;
          }
        }
      }
    }
    // fan-out tiles: few output columns, and the A instance of each output
    // instance is shared by others (or K is long enough that MFMA on
    // half-empty tiles still beats the vector units)
    V.fan = false;
    for (int t = 0; t < 2; ++t) {
      V.fanv[t].clear();
      V.n_fan[t] = 0;
    }
    if (V.kernel == 0 && nb < 5 && kb >= 3 && mb >= 6) {
      std::vector<int32_t> ua(V.ga);
      std::sort(ua.begin(), ua.end());
      const double distinct = (double)(std::unique(ua.begin(), ua.end()) - ua.begin());
      const double reuse = (double)V.ga.size() / std::max(1.0, distinct);
      if (reuse >= 2.0 || (nb == 4 && kb >= 6)) {
        // 64-column tiles when the groups are large enough to fill them
        // (the A tile is then read once for twice as many instances)
        const int tn = (nb <= 4 && reuse >= 1.5 * (double)(32 >> nb)) ? 64 : 32;
        const int order_f32[] = {0, 3, 2, -1};
        const int order_f64[] = {4, 1, -1, -1};
        const int order_h32[] = {1, 3, 2, 4};
        const int order_h64[] = {5, 0, 6, -1};
        const int* order = hm ? (tn == 64 ? order_h64 : order_h32) : (tn == 64 ? order_f64 : order_f32);
        for (int t = 0; t < 4; ++t) {
          const int c = order[t];
          const bool fits = hm ? mfma_h_fan_config_fits(c, mb, nb, kb, tn) : mfma_fan_config_fits(c, mb, nb, kb, tn);
          if (fits) {
            V.kernel = 1;
            V.fan = true;
            V.fan_tn = tn;
            V.cfg = c;
            // both tile widths' tables, so that the tuner may pick either
            make_fan(V.ga, 32 >> nb, V.fanv[0], V.n_fan[0]);
            make_fan(V.ga, 64 >> nb, V.fanv[1], V.n_fan[1]);
            const uint64_t ab = (1ull << A.idx.size()) * eb_of(P, V.swap ? V.b : V.a);
            V.fan_rows[0] = fan_block_rows(V.fanv[0], 32 >> nb, V.ga, ab);
            V.fan_rows[1] = fan_block_rows(V.fanv[1], 64 >> nb, V.ga, ab);
            break;
          }
        }
      }
    }
    if (V.kernel == 1) ++P.n_mfma;
    V.unit_rows = plain_block_units(V.ga, (1ull << A.idx.size()) * eb_of(P, V.swap ? V.b : V.a));
    V.rec_max = false;
    const double cm = std::ldexp(1.0, mb + nb + kb);
    const double w = (double)V.keys.size();
    P.cmac_single += cm;
    P.cmac_multi += w * cm;
    const double by = (double)eb_of(P, v) * w * std::ldexp(1.0, (int)V.idx.size()) +
                      (double)eb_of(P, V.swap ? V.b : V.a) * (double)A.keys.size() * std::ldexp(1.0, (int)A.idx.size()) +
                      (double)eb_of(P, V.swap ? V.a : V.b) * (double)B.keys.size() * std::ldexp(1.0, (int)B.idx.size());
    if (V.dep) {
      P.cmac_total += w * cm * nsl;
      P.bytes_slice += by;
    } else {
      P.cmac_inv += w * cm;
      P.cmac_total += w * cm;
      P.bytes_inv += by;
    }
  }
  // FP32 tensors whose maximum an FP16 consumer needs for its exponent (and
  // for the scaling of its FP16 products)
  for (int v = nt; v < P.n_nodes; ++v) {
    PNode& V = P.nodes[v];
    V.rec_max = P.precision == MATNC_CHALF && !V.half_store && V.parent >= 0 && P.nodes[V.parent].half_store;
  }
}

// offset tables of one class: entry e of level L = sum over bits t of e of
// 2^pos(index 8L+t)
void fill_table(uint32_t* T, const std::vector<int>& order, const std::vector<int>& storage) {
  std::vector<int> pos(order.size());
  for (size_t t = 0; t < order.size(); ++t) {
    auto it = std::find(storage.begin(), storage.end(), order[t]);
    pos[t] = (int)(it - storage.begin());
  }
  for (int L = 0; L < kTabLevels; ++L)
    for (int e = 0; e < kTabEntries; ++e) {
      uint32_t off = 0;
      for (int t = 0; t < 8; ++t) {
        const size_t bit = (size_t)(8 * L + t);
        if (((e >> t) & 1) && bit < pos.size()) off += 1u << pos[bit];
      }
      T[L * kTabEntries + e] = off;
    }
}

// Chunks of the reuse keys (see plan.h).  Output qubits are ordered by the
// first tree node that contains them; sorting the distinct root keys by
// their bits in that order (earliest first, most significant) puts keys
// that share the early part of the reuse tree next to each other, so a
// contiguous run of keys needs few distinct instances of the early nodes.
void build_chunks(Plan& P, int n_chunks) {
  const int nt = P.net.n_tensors;
  const int root = P.n_nodes - 1;
  const PNode& R = P.nodes[root];
  std::vector<int> first(64, INT_MAX);
  for (int v = nt; v < P.n_nodes; ++v)
    for (int q = 0; q < 64; ++q)
      if ((P.nodes[v].omask >> q) & 1) first[q] = std::min(first[q], v);
  std::vector<int> perm;
  for (int q = 0; q < 64; ++q)
    if ((R.omask >> q) & 1) perm.push_back(q);
  std::sort(perm.begin(), perm.end(), [&](int a, int b) { return first[a] != first[b] ? first[a] < first[b] : a < b; });
  auto trie = [&](uint64_t w) {
    uint64_t k = 0;
    for (size_t t = 0; t < perm.size(); ++t) k |= ((w >> perm[t]) & 1ull) << (63 - t);
    return k;
  };
  std::vector<uint64_t> rk = R.keys;
  std::sort(rk.begin(), rk.end(), [&](uint64_t a, uint64_t b) { return trie(a) < trie(b); });
  const int64_t nr = (int64_t)rk.size();
  n_chunks = (int)std::max<int64_t>(1, std::min<int64_t>(n_chunks, nr));
  P.n_chunks = n_chunks;
  P.chunks.assign(n_chunks, Chunk());
  auto find = [](const std::vector<uint64_t>& ks, uint64_t u) -> int32_t {
    return (int32_t)(std::lower_bound(ks.begin(), ks.end(), u) - ks.begin());
  };
  for (int c = 0; c < n_chunks; ++c) {
    Chunk& C = P.chunks[c];
    const int64_t lo = nr * c / n_chunks, hi = nr * (c + 1) / n_chunks;
    std::vector<uint64_t> ckeys(rk.begin() + lo, rk.begin() + hi);
    std::sort(ckeys.begin(), ckeys.end());
    // local keys of every per-batch node
    std::vector<std::vector<uint64_t>> local(P.chunked.size());
    for (size_t i = 0; i < P.chunked.size(); ++i) {
      const uint64_t m = P.nodes[P.chunked[i]].omask;
      std::vector<uint64_t>& ks = local[i];
      for (uint64_t k : ckeys) ks.push_back(k & m);
      std::sort(ks.begin(), ks.end());
      ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
    }
    C.nodes.assign(P.chunked.size(), ChunkNode());
    for (size_t i = 0; i < P.chunked.size(); ++i) {
      const int v = P.chunked[i];
      const PNode& V = P.nodes[v];
      ChunkNode& N = C.nodes[i];
      N.w = (int32_t)local[i].size();
      const int ca = V.swap ? V.b : V.a;
      const int cb = V.swap ? V.a : V.b;
      for (uint64_t u : local[i]) {
        const int pa = P.chunk_pos[ca], pb = P.chunk_pos[cb];
        const uint64_t ua = u & P.nodes[ca].omask, ub = u & P.nodes[cb].omask;
        N.ga.push_back(pa >= 0 ? find(local[pa], ua) : find(P.nodes[ca].keys, ua));
        N.gb.push_back(pb >= 0 ? find(local[pb], ub) : find(P.nodes[cb].keys, ub));
      }
      N.unit_rows = plain_block_units(N.ga, (1ull << P.nodes[ca].idx.size()) * eb_of(P, ca));
      if (V.fan) {
        const int nbits = (int)V.N.size();
        make_fan(N.ga, 32 >> nbits, N.fanv[0], N.n_fan[0]);
        make_fan(N.ga, 64 >> nbits, N.fanv[1], N.n_fan[1]);
        const uint64_t ab = (1ull << P.nodes[ca].idx.size()) * eb_of(P, ca);
        N.fan_rows[0] = fan_block_rows(N.fanv[0], 32 >> nbits, N.ga, ab);
        N.fan_rows[1] = fan_block_rows(N.fanv[1], 64 >> nbits, N.ga, ab);
      }
    }
    // rows of the batch whose root key falls in this chunk
    const int rp = P.chunk_pos[root];
    for (size_t i = 0; i < P.words.size(); ++i) {
      const uint64_t u = P.words[i] & R.omask;
      if (!std::binary_search(ckeys.begin(), ckeys.end(), u)) continue;
      C.rows.push_back((int32_t)i);
      C.rootloc.push_back(rp >= 0 ? find(local[rp], u) : find(R.keys, u));
    }
  }
}

struct ArenaBuf {
  int node;
  uint64_t size;
  int t0, t1;
};

// schedule, chunks and the static memory plan for a given chunk count
void build_memory_for(Plan& P, int n_chunks) {
  const int nt = P.net.n_tensors;
  const int root = P.n_nodes - 1;
  // schedule, each group in SSA order: the slice-invariant nodes computed
  // once per cache fill (prologue), the slice-invariant nodes computed per
  // chunk (only with several chunks: those wider than one key), and the
  // slice-dependent nodes run per slice batch (and chunk)
  P.prologue.clear();
  P.cpro.clear();
  P.loop.clear();
  for (int v = nt; v < P.n_nodes; ++v) {
    const PNode& V = P.nodes[v];
    if (V.dep)
      P.loop.push_back(v);
    else if (n_chunks > 1 && V.keys.size() > 1)
      P.cpro.push_back(v);
    else
      P.prologue.push_back(v);
  }
  P.chunked = P.cpro;
  P.chunked.insert(P.chunked.end(), P.loop.begin(), P.loop.end());
  P.chunk_pos.assign(P.n_nodes, -1);
  for (size_t i = 0; i < P.chunked.size(); ++i) P.chunk_pos[P.chunked[i]] = (int)i;
  build_chunks(P, n_chunks);
  int t = 0;
  for (int v : P.prologue) P.nodes[v].time = t++;
  for (int v : P.chunked) P.nodes[v].time = t++;
  const int t_end = t + 1;
  // instance capacity of every node: the largest chunk
  std::vector<int64_t> cap_inst(P.n_nodes, 0);
  for (int v = 0; v < P.n_nodes; ++v) cap_inst[v] = (int64_t)P.nodes[v].keys.size();
  for (size_t i = 0; i < P.chunked.size(); ++i) {
    int64_t mx = 0;
    for (const Chunk& C : P.chunks) mx = std::max<int64_t>(mx, C.nodes[i].w);
    cap_inst[P.chunked[i]] = mx;
  }

  // static region
  uint64_t off = 0;
  P.sigma_off = off;
  off += kAlign;
  for (int v = nt; v < P.n_nodes; ++v) {
    PNode& V = P.nodes[v];
    V.tab_off = off;
    off = align_up(off + (uint64_t)TAB_COUNT * kTabSize * 4);
    if (P.chunk_pos[v] < 0) {
      V.ga_off = off;
      off = align_up(off + V.ga.size() * 4);
      V.gb_off = off;
      off = align_up(off + V.gb.size() * 4);
      for (int t = 0; t < 2; ++t) {
        V.fan_off[t] = off;
        off = align_up(off + V.fanv[t].size() * 4);
      }
    }
  }
  // per-chunk index lists, packed back to back (int32 entries)
  for (Chunk& C : P.chunks) {
    for (ChunkNode& N : C.nodes) {
      N.ga_off = off;
      off += N.ga.size() * 4;
      N.gb_off = off;
      off += N.gb.size() * 4;
      for (int t = 0; t < 2; ++t) {
        N.fan_off[t] = off;
        off += N.fanv[t].size() * 4;
      }
    }
    C.rows_off = off;
    off += C.rows.size() * 4;
    C.rootloc_off = off;
    off += C.rootloc.size() * 4;
  }
  off = align_up(off);
  // leaf variants: keys x 2^nsb instances
  for (int l = 0; l < nt; ++l) {
    PNode& L = P.nodes[l];
    L.inst_elems = 1ull << L.idx.size();
    L.off = off;
    L.buf_bytes = (uint64_t)L.keys.size() * (1ull << L.sl_bits.size()) * L.inst_elems * 8;
    off = align_up(off + L.buf_bytes);
  }
  if (P.precision == MATNC_CHALF) {
    const uint64_t hs = sizeof(HalfScale);
    for (int l = 0; l < nt; ++l) {
      PNode& L = P.nodes[l];
      L.scale_off = off;
      off = align_up(off + (uint64_t)L.keys.size() * (1ull << L.sl_bits.size()) * hs);
    }
    P.inv_scale_lo = off;
    for (int v : P.prologue) {
      P.nodes[v].scale_off = off;
      off += (uint64_t)P.nodes[v].keys.size() * hs;
    }
    off = align_up(off);
    P.inv_scale_hi = off;
    P.cpro_scale_lo = off;
    for (int v : P.cpro) {
      P.nodes[v].scale_off = off;
      off += (uint64_t)cap_inst[v] * hs;
    }
    off = align_up(off);
    P.cpro_scale_hi = off;
    P.dep_scale_lo = off;
    for (int v : P.loop) {
      P.nodes[v].scale_off = off;
      off += (uint64_t)cap_inst[v] * P.batch * hs;
    }
    off = align_up(off);
    P.dep_scale_hi = off;
  }
  P.static_bytes = off;

  // intermediates
  std::vector<ArenaBuf> bufs;
  for (int v = nt; v < P.n_nodes; ++v) {
    PNode& V = P.nodes[v];
    V.inst_elems = 1ull << V.idx.size();
    const uint64_t ninst = (uint64_t)cap_inst[v] * (V.dep ? (uint64_t)P.batch : 1ull);
    V.buf_bytes = align_up(ninst * V.inst_elems * eb_of(P, v));
    const PNode& Par = P.nodes[v == root ? root : V.parent];
    int t1;
    if (v == root)
      t1 = t_end;
    else if (!V.dep && Par.dep)
      t1 = t_end;  // cache: read by every slice batch (of its chunk)
    else if (P.chunk_pos[v] < 0 && P.chunk_pos[V.parent] >= 0)
      t1 = t_end;  // prologue result read by every chunk
    else
      t1 = Par.time;
    bufs.push_back({v, V.buf_bytes, V.time, t1});
  }
  std::sort(bufs.begin(), bufs.end(), [](const ArenaBuf& x, const ArenaBuf& y) {
    return x.size != y.size ? x.size > y.size : x.t0 < y.t0;
  });
  std::vector<std::pair<uint64_t, uint64_t>> placed_range;  // per placed buf
  std::vector<const ArenaBuf*> placed;
  uint64_t arena = 0;
  P.cache_bytes = 0;
  for (const ArenaBuf& b : bufs) {
    std::vector<std::pair<uint64_t, uint64_t>> busy;
    for (size_t i = 0; i < placed.size(); ++i)
      if (!(placed[i]->t1 < b.t0 || b.t1 < placed[i]->t0)) busy.push_back(placed_range[i]);
    std::sort(busy.begin(), busy.end());
    uint64_t cur = 0;
    for (auto& r : busy) {
      if (r.first >= cur + b.size) break;
      cur = std::max(cur, r.second);
    }
    placed.push_back(&b);
    placed_range.push_back({cur, cur + b.size});
    P.nodes[b.node].off = P.static_bytes + cur;
    arena = std::max(arena, cur + b.size);
    if (b.t1 == t_end && b.node != root) P.cache_bytes += b.size;
  }
  P.workspace_bytes = align_up(P.static_bytes + arena);
}

// smallest power-of-two chunk count whose workspace fits the budget
void build_memory(Plan& P) {
  int c = 1;
  build_memory_for(P, c);
  const int64_t nr = (int64_t)P.nodes[P.n_nodes - 1].keys.size();
  while (P.memory_budget && P.workspace_bytes > P.memory_budget && c < nr) {
    c *= 2;
    build_memory_for(P, c);
  }
  if (P.memory_budget && P.workspace_bytes > P.memory_budget)
    fail(MATNC_E_NOMEM, "plan needs " + std::to_string(P.workspace_bytes) + " bytes of workspace even with " +
                            std::to_string(P.n_chunks) + " key chunks; budget " + std::to_string(P.memory_budget));
}

// writes leaf l's variants (and, for complex-half, its scales) into the
// static-region image dst (indexed by workspace offsets)
void fill_leaf_data(Plan& P, int l, unsigned char* dst) {
  const Network& N = P.net;
  const PNode& L = P.nodes[l];
  const std::vector<int>& ix = N.idx[l];
  const int r = (int)ix.size();
  std::unordered_map<int, int> out_qubit;
  for (int q = 0; q < N.n_qubits; ++q) out_qubit[N.out_index[q]] = q;
  // role of each original axis
  std::vector<int> kind(r), arg(r);  // 0 closed output (qubit), 1 sliced (t), 2 free (pos)
  for (int a = 0; a < r; ++a) {
    const int i = ix[a];
    auto fp = std::find(L.idx.begin(), L.idx.end(), i);
    if (fp != L.idx.end()) {
      kind[a] = 2;
      arg[a] = (int)(fp - L.idx.begin());
      continue;
    }
    auto sp = std::find(L.sl_index.begin(), L.sl_index.end(), i);
    if (sp != L.sl_index.end()) {
      kind[a] = 1;
      arg[a] = (int)(sp - L.sl_index.begin());
      continue;
    }
    kind[a] = 0;
    arg[a] = out_qubit.at(i);
  }
  const uint64_t nsv = 1ull << L.sl_bits.size();
  const uint64_t ne = L.inst_elems;
  const std::vector<double>& src = N.data[l];
  uint64_t inst = 0;
  for (size_t u = 0; u < L.keys.size(); ++u) {
    for (uint64_t sv = 0; sv < nsv; ++sv, ++inst) {
      float smx = 0.f;
      for (uint64_t e = 0; e < ne; ++e) {
        uint64_t flat = 0;
        for (int a = 0; a < r; ++a) {
          uint64_t bit;
          if (kind[a] == 0)
            bit = (L.keys[u] >> arg[a]) & 1;
          else if (kind[a] == 1)
            bit = (sv >> arg[a]) & 1;
          else
            bit = (e >> arg[a]) & 1;
          flat |= bit << (r - 1 - a);
        }
        const double re = src[2 * flat], im = src[2 * flat + 1];
        const uint64_t d = inst * ne + e;
        float* f = reinterpret_cast<float*>(dst + L.off) + 2 * d;
        f[0] = (float)re;
        f[1] = (float)im;
        smx = std::max(smx, std::max(std::fabs(f[0]), std::fabs(f[1])));
      }
      if (P.precision == MATNC_CHALF) {
        // leaves stay FP32 (exponent 0); their maximum feeds the scale
        // choice of FP16 consumers
        HalfScale hs;
        hs.e = 0;
        std::memcpy(&hs.mx, &smx, 4);
        std::memcpy(dst + L.scale_off + inst * sizeof(HalfScale), &hs, sizeof(hs));
      }
    }
  }
}

// how a node of chunk c reads child `child` (gmap_off: the gather map)
OpDesc operand_desc(const Plan& P, int child, uint64_t gmap_off, int c) {
  const PNode& C = P.nodes[child];
  OpDesc o;
  std::memset(&o, 0, sizeof(o));
  o.off = C.off + (child >= P.net.n_tensors ? P.arena_delta : 0);
  o.inst_bytes = C.inst_elems * eb_of(P, child);
  o.half = C.half_store ? 1 : 0;
  o.gmap_off = gmap_off;
  o.scale_off = C.scale_off;
  const int pos = P.chunk_pos.empty() ? -1 : P.chunk_pos[child];
  o.w_child = pos >= 0 ? P.chunks[c].nodes[pos].w : (int32_t)C.keys.size();
  const bool leaf = child < P.net.n_tensors;
  o.dep = (!leaf && C.dep) ? 1 : 0;
  o.nsb = leaf ? (int32_t)C.sl_bits.size() : 0;
  o.nsv = 1 << o.nsb;
  for (int t = 0; t < o.nsb; ++t) o.sbit[t] = (int8_t)C.sl_bits[t];
  return o;
}

NodeDesc node_desc(const Plan& P, int v, int nb, int c = 0) {
  const PNode& V = P.nodes[v];
  NodeDesc d;
  std::memset(&d, 0, sizeof(d));
  const int ca = V.swap ? V.b : V.a;
  const int cb = V.swap ? V.a : V.b;
  const int pos = P.chunk_pos[v];
  const uint64_t ga = pos >= 0 ? P.chunks[c].nodes[pos].ga_off : V.ga_off;
  const uint64_t gb = pos >= 0 ? P.chunks[c].nodes[pos].gb_off : V.gb_off;
  d.A = operand_desc(P, ca, ga, c);
  d.B = operand_desc(P, cb, gb, c);
  d.c_off = V.off + P.arena_delta;
  d.c_inst_bytes = V.inst_elems * eb_of(P, v);
  d.c_half = V.half_store ? 1 : 0;
  d.tab_off = V.tab_off;
  d.c_scale_off = V.scale_off;
  d.w = pos >= 0 ? P.chunks[c].nodes[pos].w : (int32_t)V.keys.size();
  d.dep = V.dep ? 1 : 0;
  d.n_inst = (int64_t)d.w * (V.dep ? nb : 1);
  d.mbits = (int32_t)V.M.size();
  d.nbits = (int32_t)V.N.size();
  d.kbits = (int32_t)V.K.size();
  if (V.fan) {
    const int t = V.fan_tn == 64 ? 1 : 0;
    d.fan_off = pos >= 0 ? P.chunks[c].nodes[pos].fan_off[t] : V.fan_off[t];
    d.n_fan = pos >= 0 ? P.chunks[c].nodes[pos].n_fan[t] : V.n_fan[t];
    d.fan_tn = V.fan_tn;
    d.fan_rows = pos >= 0 ? P.chunks[c].nodes[pos].fan_rows[t] : V.fan_rows[t];
  } else {
    d.fan_rows = pos >= 0 ? P.chunks[c].nodes[pos].unit_rows : V.unit_rows;
  }
  return d;
}

// the root as read by the slice-sum of chunk c: instance per row position
OpDesc root_desc(const Plan& P, int c) {
  const int root = P.n_nodes - 1;
  return operand_desc(P, root, P.chunks[c].rootloc_off, c);
}

// Queue plans that share an arena: before launching into it, a plan takes
// it over; if another plan held it, this plan's stem cache is gone.
void claim_arena(Plan& P) {
  if (!P.share) return;
  if (P.share->owner != P.share_id) P.inv_valid = false;
  P.share->owner = P.share_id;
}

void launch_node(const Plan& P, const PNode& V, const NodeDesc& d, hipStream_t st) {
  const int64_t* sig = reinterpret_cast<const int64_t*>(P.ws + P.sigma_off);
  hipError_t e;
  if (V.kernel == 1 && !V.half_store) {
    // FP32 MFMA (an FP16-stored operand is widened exactly as it is loaded);
    // an FP16 consumer's scaling needs the output maxima: fan-out
    // tiles record them in their epilogue, other tiles leave them to a
    // separate reduction pass (recording in the epilogue of the big tiles
    // raises their register use and cuts the occupancy)
    if (V.fan) {
      e = V.rec_max ? launch_mfma_fan_rec(d, V.cfg, P.ws, sig, st) : launch_mfma_fan(d, V.cfg, P.ws, sig, st);
    } else {
      e = launch_mfma(d, V.cfg, P.ws, sig, st);
      if (e == hipSuccess && V.rec_max) e = launch_absmax(d, P.ws, st);
    }
  } else if (V.kernel == 1) {
    e = V.fan ? launch_mfma_h_fan(d, V.cfg, P.ws, sig, st) : launch_mfma_h(d, V.cfg, P.ws, sig, st);
  } else if (P.precision == MATNC_C64) {
    e = launch_stream(d, P.ws, sig, st);
  } else {
    // steps with no FP16 operand or output and whose maximum nobody reads
    // take the complex64 kernels
    e = (V.half_store || V.rec_max || d.A.half || d.B.half) ? launch_stream_h(d, P.ws, sig, st)
                                                             : launch_stream(d, P.ws, sig, st);
  }
  hip_check(e, "kernel launch");
}

// one slice batch of chunk c: the per-batch nodes, then the slice-sum of
// the chunk's rows into amps (skipped when amps is null)
// HIP events around every launch of one node (the rest run as usual)
struct StepTimer {
  int v = -1;
  std::vector<hipEvent_t> ev;  // (begin, end) pairs, one per launch
  ~StepTimer() {
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

void launch_node_timed(const Plan& P, int v, const NodeDesc& d, hipStream_t st, StepTimer* t) {
  if (!t || v != t->v) {
    launch_node(P, P.nodes[v], d, st);
    return;
  }
  for (int i = 0; i < 2; ++i) {
    t->ev.push_back(nullptr);
    hip_check(hipEventCreate(&t->ev.back()), "event create");
  }
  const size_t n = t->ev.size();
  hip_check(hipEventRecord(t->ev[n - 2], st), "event record");
  launch_node(P, P.nodes[v], d, st);
  hip_check(hipEventRecord(t->ev[n - 1], st), "event record");
}

void launch_batch(const Plan& P, int c, int nb, hipStream_t st, double* amps, StepTimer* t = nullptr) {
  const int64_t* sig = reinterpret_cast<const int64_t*>(P.ws + P.sigma_off);
  const int ob = (int)P.open_qubits.size();
  if (P.precision == MATNC_CHALF)
    hip_check(launch_zero(P.ws + P.dep_scale_lo, P.dep_scale_hi - P.dep_scale_lo, st), "clear scales");
  for (int v : P.loop) launch_node_timed(P, v, node_desc(P, v, nb, c), st, t);
  if (!amps) return;
  const Chunk& C = P.chunks[c];
  const OpDesc root = root_desc(P, c);
  const int64_t nrows = (int64_t)C.rows.size();
  const int32_t* rows = reinterpret_cast<const int32_t*>(P.ws + C.rows_off);
  hipError_t er = P.precision == MATNC_C64 ? launch_slice_sum(root, P.ws, sig, nb, nrows, rows, ob, amps, st)
                                           : launch_slice_sum_h(root, P.ws, sig, nb, nrows, rows, ob, amps, st);
  hip_check(er, "slice sum");
}

void launch_prologue(const Plan& P, hipStream_t st, StepTimer* t = nullptr) {
  if (P.precision == MATNC_CHALF)
    hip_check(launch_zero(P.ws + P.inv_scale_lo, P.inv_scale_hi - P.inv_scale_lo, st), "clear scales");
  for (int v : P.prologue) launch_node_timed(P, v, node_desc(P, v, 1), st, t);
}

// chunk c's instances of the per-chunk invariant nodes
void launch_chunk_prologue(const Plan& P, int c, hipStream_t st, StepTimer* t = nullptr) {
  if (P.cpro.empty()) return;
  if (P.precision == MATNC_CHALF)
    hip_check(launch_zero(P.ws + P.cpro_scale_lo, P.cpro_scale_hi - P.cpro_scale_lo, st), "clear scales");
  for (int v : P.cpro) launch_node_timed(P, v, node_desc(P, v, 1, c), st, t);
}

void release_graph(Plan& P) {
  for (auto g : P.graph_execs)
    if (g) (void)hipGraphExecDestroy(g);
  for (auto g : P.graphs)
    if (g) (void)hipGraphDestroy(g);
  P.graph_execs.clear();
  P.graphs.clear();
  P.graph_amps = nullptr;
}

// capture one full slice batch of every chunk (adding into amps) as graphs;
// not possible on the null stream
void capture_batch_graphs(Plan& P, double* amps) {
  release_graph(P);
  if (P.stream == nullptr || amps == nullptr) return;
  for (int c = 0; c < P.n_chunks; ++c) {
    hip_check(hipStreamBeginCapture(P.stream, hipStreamCaptureModeThreadLocal), "begin capture");
    hipGraph_t g = nullptr;
    try {
      launch_batch(P, c, P.batch, P.stream, amps);
    } catch (...) {
      (void)hipStreamEndCapture(P.stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    hip_check(hipStreamEndCapture(P.stream, &g), "end capture");
    P.graphs.push_back(g);
    hipGraphExec_t x = nullptr;
    hip_check(hipGraphInstantiate(&x, g, nullptr, nullptr, 0), "graph instantiate");
    P.graph_execs.push_back(x);
  }
  P.graph_amps = amps;
}

// every launch of a complete pass over slices [b, e) into amps (no graphs)
void launch_pass(Plan& P, int64_t b, int64_t e, double* amps, hipStream_t st) {
  int64_t* sig = reinterpret_cast<int64_t*>(P.ws + P.sigma_off);
  hip_check(launch_set_i64(sig, 0, st), "set sigma");
  launch_prologue(P, st);
  for (int c = 0; c < P.n_chunks; ++c) {
    launch_chunk_prologue(P, c, st);
    for (int64_t s0 = b; s0 < e; s0 += P.batch) {
      const int nb = (int)std::min<int64_t>(P.batch, e - s0);
      hip_check(launch_set_i64(sig, s0, st), "set sigma");
      launch_batch(P, c, nb, st, amps);
    }
  }
}

// shape class of an MFMA step for the tuning cache
std::string tune_key(const Plan& P, const PNode& V, int64_t n_inst) {
  int lg = 0;
  while ((1LL << lg) < n_inst) ++lg;
  return std::string(P.precision == MATNC_C64 ? "c64" : "chalf") + (V.half_store ? "/h" : "/f") +
         (V.fan ? "/fan" : "") + "/" +
         std::to_string(V.M.size()) + "," + std::to_string(V.N.size()) + "," + std::to_string(V.K.size()) + "/" +
         std::to_string(lg);
}

std::map<std::string, int> read_tune_cache(const char* path) {
  std::map<std::string, int> out;
  if (!path) return out;
  FILE* f = std::fopen(path, "r");
  if (!f) return out;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
  std::fclose(f);
  // entries "key": integer
  size_t pos = 0;
  while ((pos = text.find('"', pos)) != std::string::npos) {
    const size_t end = text.find('"', pos + 1);
    if (end == std::string::npos) break;
    const std::string key = text.substr(pos + 1, end - pos - 1);
    const size_t colon = text.find(':', end);
    if (colon == std::string::npos) break;
    out[key] = std::atoi(text.c_str() + colon + 1);
    pos = colon + 1;
  }
  return out;
}

void write_tune_cache(const char* path, const std::map<std::string, int>& m) {
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) fail(MATNC_E_INVALID, std::string("cannot write tuning cache ") + path);
  std::fprintf(f, "{\n");
  size_t i = 0;
  for (auto& kv : m) std::fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++i < m.size() ? "," : "");
  std::fprintf(f, "}\n");
  std::fclose(f);
  if (std::rename(tmp.c_str(), path) != 0) fail(MATNC_E_INVALID, std::string("cannot write tuning cache ") + path);
}

// ---------------------------------------------------------------------------
// single pairwise contractions (matnc_contract, matnc_contract_noalloc)

// scratch of one call: a zero head (int64 sigma slot at byte 0, a zero
// int32 gather entry at byte 8), then the six offset tables
constexpr size_t kContractScratchBytes = kAlign + (size_t)TAB_COUNT * kTabSize * 4;

struct TabPos {
  int8_t pos[TAB_COUNT][32];  // storage bit of coordinate bit i, per table class
  int32_t nbits[TAB_COUNT];
};

struct ContractCall {
  int64_t batch;
  int nm, nn, nk;
  int kind, cfg;  // 0 streaming, 1 MFMA configuration cfg
  TabPos pos;
};

// validates the arguments of one contraction and picks its kernel
ContractCall contract_call(int64_t batch, int nm, int nn, int nk, const int* posA_m, const int* posA_k,
                           const int* posB_k, const int* posB_n, const int* posC_m, const int* posC_n, int kernel) {
  if (batch < 0) fail(MATNC_E_INVALID, "batch must be >= 0");
  if (nm < 0 || nn < 0 || nk < 0 || nm + nk > 32 || nn + nk > 32 || nm + nn > 32)
    fail(MATNC_E_INVALID, "ranks must be <= 32");
  if ((nm && (!posA_m || !posC_m)) || (nn && (!posB_n || !posC_n)) || (nk && (!posA_k || !posB_k)))
    fail(MATNC_E_INVALID, "null position array");
  auto check_perm = [](std::vector<int> p, const char* what) {
    std::sort(p.begin(), p.end());
    for (size_t i = 0; i < p.size(); ++i)
      if (p[i] != (int)i) fail(MATNC_E_INVALID, std::string(what) + " positions are not a permutation");
  };
  std::vector<int> pa, pb, pc;
  for (int t = 0; t < nm; ++t) pa.push_back(posA_m[t]);
  for (int t = 0; t < nk; ++t) pa.push_back(posA_k[t]);
  for (int t = 0; t < nk; ++t) pb.push_back(posB_k[t]);
  for (int t = 0; t < nn; ++t) pb.push_back(posB_n[t]);
  for (int t = 0; t < nm; ++t) pc.push_back(posC_m[t]);
  for (int t = 0; t < nn; ++t) pc.push_back(posC_n[t]);
  check_perm(pa, "A");
  check_perm(pb, "B");
  check_perm(pc, "C");
  ContractCall c;
  std::memset(&c, 0, sizeof(c));
  c.batch = batch;
  c.nm = nm;
  c.nn = nn;
  c.nk = nk;
  c.kind = 0;
  c.cfg = -1;
  if (kernel == -1) {
    if (nn + nk > 8) {
      const int order[] = {1, 0, 3, 2};
      for (int k : order)
        if (mfma_config_fits(k, nm, nn, nk)) {
          c.kind = 1;
          c.cfg = k;
          break;
        }
    }
  } else if (kernel == 0) {
    c.kind = 0;
  } else if (kernel == 1) {
    for (int k = 0; k < mfma_config_count() && c.cfg < 0; ++k)
      if (mfma_config_fits(k, nm, nn, nk)) c.cfg = k;
    if (c.cfg < 0) fail(MATNC_E_INVALID, "no MFMA tile fits this shape");
    c.kind = 1;
  } else if (kernel >= 100 && kernel < 100 + mfma_config_count()) {
    c.cfg = kernel - 100;
    if (!mfma_config_fits(c.cfg, nm, nn, nk)) fail(MATNC_E_INVALID, "MFMA tile does not fit this shape");
    c.kind = 1;
  } else {
    fail(MATNC_E_INVALID, "unknown kernel selector");
  }
  const int* src[TAB_COUNT];
  src[TAB_AM] = posA_m;
  src[TAB_CM] = posC_m;
  src[TAB_BN] = posB_n;
  src[TAB_CN] = posC_n;
  src[TAB_AK] = posA_k;
  src[TAB_BK] = posB_k;
  const int nb[TAB_COUNT] = {nm, nm, nn, nn, nk, nk};
  for (int t = 0; t < TAB_COUNT; ++t) {
    c.pos.nbits[t] = nb[t];
    for (int i = 0; i < nb[t]; ++i) c.pos.pos[t][i] = (int8_t)src[t][i];
  }
  return c;
}

// the contraction of one call; base = device address of its scratch
void launch_contract(const ContractCall& c, const void* A, const void* B, void* C, uint64_t base, hipStream_t st) {
  NodeDesc d;
  std::memset(&d, 0, sizeof(d));
  auto op = [&](const void* p, int rank) {
    OpDesc o;
    std::memset(&o, 0, sizeof(o));
    o.off = reinterpret_cast<uint64_t>(p);
    o.inst_bytes = 8ull << rank;
    o.gmap_off = base + 8;  // a single zero entry
    o.w_child = 1;
    o.dep = 1;
    o.nsv = 1;
    return o;
  };
  d.A = op(A, c.nm + c.nk);
  d.B = op(B, c.nn + c.nk);
  d.c_off = reinterpret_cast<uint64_t>(C);
  d.c_inst_bytes = 8ull << (c.nm + c.nn);
  d.tab_off = base + kAlign;
  d.w = 1;
  d.dep = 1;
  d.n_inst = c.batch;
  d.mbits = c.nm;
  d.nbits = c.nn;
  d.kbits = c.nk;
  const int64_t* sig = reinterpret_cast<const int64_t*>(base);
  hipError_t e = c.kind == 1 ? launch_mfma(d, c.cfg, 0, sig, st) : launch_stream(d, 0, sig, st);
  hip_check(e, "contract launch");
}

// The scratch of matnc_contract_noalloc: one copy per GPU, held until the
// process ends, shared by every call on that GPU (calls that overlap on one
// GPU race on it).  Host code never uses the symbol's name as an address:
// the device address of each GPU's copy comes from hipGetSymbolAddress,
// taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[32768];

__global__ void k_contract_tables(TabPos pos, uint32_t* base) {
  // block t writes table class t; block 0 also clears the head (sigma slot
  // and the zero gather entry)
  const int t = blockIdx.x, e = threadIdx.x;
  if (t == 0 && e < (int)(kAlign / 4)) base[e] = 0u;
  uint32_t* T = base + kAlign / 4 + t * kTabSize;
  for (int L = 0; L < kTabLevels; ++L) {
    uint32_t off = 0;
    for (int b = 0; b < 8; ++b) {
      const int bit = 8 * L + b;
      if (((e >> b) & 1) && bit < pos.nbits[t]) off += 1u << pos.pos[t][bit];
    }
    T[L * kTabEntries + e] = off;
  }
}

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_dev;  // device address of `scratch` per device id

void* static_scratch_ptr() {
  int dev = 0;
  hip_check(hipGetDevice(&dev), "get device");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((size_t)dev >= g_scratch_dev.size()) g_scratch_dev.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch symbol address");
    if (!p) fail(MATNC_E_HIP, "scratch symbol has no device address");
    g_scratch_dev[dev] = p;
  }
  return g_scratch_dev[dev];
}

// attaches plan P to its static region at dev_workspace (and its arena at
// dev_workspace + static_bytes + arena_delta), uploads the static region
void bind_plan(Plan& P, void* dev_workspace, size_t bytes, void* hip_stream, uint64_t arena_delta,
               std::shared_ptr<ArenaShare> share) {
  release_graph(P);
  P.bound = false;
  P.ws = reinterpret_cast<uint64_t>(dev_workspace);
  P.ws_bytes = bytes;
  P.arena_delta = arena_delta;
  P.share = std::move(share);
  if (P.share) {
    static std::atomic<uint64_t> next_id{0};
    P.share_id = ++next_id;
  }
  P.stream = reinterpret_cast<hipStream_t>(hip_stream);
  // host image of the static region
  P.staging.assign(P.static_bytes, 0);
  const int nt = P.net.n_tensors;
  for (int v = nt; v < P.n_nodes; ++v) {
    const PNode& V = P.nodes[v];
    uint32_t* T = reinterpret_cast<uint32_t*>(P.staging.data() + V.tab_off);
    const PNode& A = P.nodes[V.swap ? V.b : V.a];
    const PNode& B = P.nodes[V.swap ? V.a : V.b];
    fill_table(T + TAB_AM * kTabSize, V.M, A.idx);
    fill_table(T + TAB_CM * kTabSize, V.M, V.idx);
    fill_table(T + TAB_BN * kTabSize, V.N, B.idx);
    fill_table(T + TAB_CN * kTabSize, V.N, V.idx);
    fill_table(T + TAB_AK * kTabSize, V.K, A.idx);
    fill_table(T + TAB_BK * kTabSize, V.K, B.idx);
    if (P.chunk_pos[v] < 0) {
      std::memcpy(P.staging.data() + V.ga_off, V.ga.data(), V.ga.size() * 4);
      std::memcpy(P.staging.data() + V.gb_off, V.gb.data(), V.gb.size() * 4);
      for (int t = 0; t < 2; ++t)
        std::memcpy(P.staging.data() + V.fan_off[t], V.fanv[t].data(), V.fanv[t].size() * 4);
    }
  }
  for (const Chunk& C : P.chunks) {
    for (const ChunkNode& N : C.nodes) {
      std::memcpy(P.staging.data() + N.ga_off, N.ga.data(), N.ga.size() * 4);
      std::memcpy(P.staging.data() + N.gb_off, N.gb.data(), N.gb.size() * 4);
      for (int t = 0; t < 2; ++t)
        std::memcpy(P.staging.data() + N.fan_off[t], N.fanv[t].data(), N.fanv[t].size() * 4);
    }
    std::memcpy(P.staging.data() + C.rows_off, C.rows.data(), C.rows.size() * 4);
    std::memcpy(P.staging.data() + C.rootloc_off, C.rootloc.data(), C.rootloc.size() * 4);
  }
  for (int l = 0; l < nt; ++l) fill_leaf_data(P, l, P.staging.data());
  hip_check(hipMemcpyAsync(dev_workspace, P.staging.data(), P.static_bytes, hipMemcpyHostToDevice, P.stream),
            "upload static region");
  hip_check(hipStreamSynchronize(P.stream), "upload static region");
  P.bound = true;
  P.inv_valid = false;
  ++P.generation;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char* matnc_version(void) { return "matnc 0.1.0 gfx950"; }

const char* matnc_last_error(void) { return g_err.c_str(); }

int matnc_network_create(int n_tensors, const int* ranks, const int* index_ids, const double* data_c128,
                         int n_qubits, const int* output_index_of_qubit, matnc_network* out) {
  return guarded([&] {
    if (!out || !ranks || !index_ids || !data_c128 || !output_index_of_qubit)
      fail(MATNC_E_INVALID, "null argument");
    if (n_tensors < 1) fail(MATNC_E_INVALID, "n_tensors must be >= 1");
    if (n_qubits < 1 || n_qubits > 64) fail(MATNC_E_INVALID, "n_qubits must be in 1..64");
    auto h = new matnc_network_s();
    std::unique_ptr<matnc_network_s> guard(h);
    Network& N = h->net;
    N.n_tensors = n_tensors;
    N.n_qubits = n_qubits;
    N.idx.resize(n_tensors);
    N.data.resize(n_tensors);
    size_t ip = 0, dp = 0;
    std::unordered_map<int, int> count;
    for (int t = 0; t < n_tensors; ++t) {
      const int r = ranks[t];
      if (r < 0 || r > 20) fail(MATNC_E_INVALID, "tensor rank must be in 0..20");
      N.idx[t].assign(index_ids + ip, index_ids + ip + r);
      ip += r;
      std::vector<int> s = N.idx[t];
      std::sort(s.begin(), s.end());
      if (std::adjacent_find(s.begin(), s.end()) != s.end())
        fail(MATNC_E_INVALID, "tensor " + std::to_string(t) + " repeats an index");
      for (int i : s) {
        if (i < 0) fail(MATNC_E_INVALID, "index ids must be >= 0");
        ++count[i];
      }
      const size_t ne = (size_t)1 << r;
      N.data[t].assign(data_c128 + 2 * dp, data_c128 + 2 * (dp + ne));
      dp += ne;
    }
    N.out_index.assign(output_index_of_qubit, output_index_of_qubit + n_qubits);
    std::unordered_map<int, int> seen_out;
    for (int q = 0; q < n_qubits; ++q) {
      const int i = N.out_index[q];
      if (seen_out.count(i)) fail(MATNC_E_INVALID, "two qubits share an output index");
      seen_out[i] = q;
      if (count[i] != 1) fail(MATNC_E_INVALID, "output index of qubit " + std::to_string(q) + " must occur once");
    }
    for (auto& kv : count)
      if (!seen_out.count(kv.first) && kv.second != 2)
        fail(MATNC_E_INVALID, "index " + std::to_string(kv.first) + " occurs " + std::to_string(kv.second) +
                                  " times (bond indices occur on exactly two tensors)");
    *out = guard.release();
  });
}

int matnc_network_destroy(matnc_network net) {
  delete net;
  return MATNC_OK;
}

int matnc_plan_create(matnc_network net, const int* pairs, int n_sliced, const int* sliced_ids, int n_open,
                      const int* open_qubits, int64_t k, const uint64_t* bitstrings, int precision, int max_rank,
                      int slice_batch, size_t memory_budget, matnc_plan* out) {
  matnc_plan_options_t o;
  std::memset(&o, 0, sizeof(o));
  o.slice_batch = slice_batch;
  o.memory_budget = memory_budget;
  o.half_nodes = -1;
  return matnc_plan_create_ex(net, pairs, n_sliced, sliced_ids, n_open, open_qubits, k, bitstrings, precision,
                              max_rank, &o, out);
}

int matnc_plan_create_ex(matnc_network net, const int* pairs, int n_sliced, const int* sliced_ids, int n_open,
                         const int* open_qubits, int64_t k, const uint64_t* bitstrings, int precision, int max_rank,
                         const matnc_plan_options_t* opts, matnc_plan* out) {
  return guarded([&] {
    if (!opts) fail(MATNC_E_INVALID, "null options");
    const int slice_batch = opts->slice_batch;
    const size_t memory_budget = opts->memory_budget;
    if (opts->half_nodes < -1) fail(MATNC_E_INVALID, "half_nodes must be >= -1");
    if (!net || !out) fail(MATNC_E_INVALID, "null argument");
    const Network& N = net->net;
    const int nt = N.n_tensors;
    if (nt > 1 && !pairs) fail(MATNC_E_INVALID, "null pairs");
    if (n_sliced < 0 || n_sliced > 40) fail(MATNC_E_INVALID, "n_sliced must be in 0..40");
    if (n_sliced > 0 && !sliced_ids) fail(MATNC_E_INVALID, "null sliced_ids");
    if (n_open < 0 || n_open > N.n_qubits || n_open > 24) fail(MATNC_E_INVALID, "n_open must be in 0..min(n,24)");
    if (n_open > 0 && !open_qubits) fail(MATNC_E_INVALID, "null open_qubits");
    if (k < 1 || k > (int64_t)1 << 31 || !bitstrings) fail(MATNC_E_INVALID, "k must be in 1..2^31");
    if (precision != MATNC_C64 && precision != MATNC_CHALF) fail(MATNC_E_INVALID, "unknown precision");
    if (precision == MATNC_CHALF && !chalf_available()) fail(MATNC_E_INVALID, "complex-half path not built");
    if (max_rank < 0) fail(MATNC_E_INVALID, "max_rank must be >= 0");
    if (slice_batch < 1) fail(MATNC_E_INVALID, "slice_batch must be >= 1");
    auto h = new matnc_plan_s();
    std::unique_ptr<matnc_plan_s> guard(h);
    Plan& P = h->p;
    P.net = N;
    P.precision = precision;
    P.elem_bytes = precision == MATNC_C64 ? 8 : 4;
    P.max_rank_cap = max_rank;
    P.batch = slice_batch;
    P.memory_budget = memory_budget;
    const int64_t n_amps = k << n_open;
    P.half_nodes = opts->half_nodes >= 0 ? opts->half_nodes
                                         : (int)std::min<int64_t>(kMaxHalfNodes, n_amps / kAmpsPerHalfNode);
    // tree
    std::vector<char> used(2 * nt - 1, 0);
    for (int j = 0; j < nt - 1; ++j) {
      const int a = pairs[2 * j], b = pairs[2 * j + 1];
      if (a < 0 || b < 0 || a >= nt + j || b >= nt + j || a == b || used[a] || used[b])
        fail(MATNC_E_INVALID, "pairs do not form a contraction tree (step " + std::to_string(j) + ")");
      used[a] = used[b] = 1;
      P.pairs.push_back({a, b});
    }
    // sliced indices: bond indices, distinct
    std::unordered_map<int, int> count;
    for (auto& ix : N.idx)
      for (int i : ix) ++count[i];
    std::unordered_map<int, int> outs;
    for (int q = 0; q < N.n_qubits; ++q) outs[N.out_index[q]] = q;
    for (int j = 0; j < n_sliced; ++j) {
      const int i = sliced_ids[j];
      if (outs.count(i) || count[i] != 2) fail(MATNC_E_INVALID, "sliced id " + std::to_string(i) + " is not a bond");
      if (std::find(P.sliced.begin(), P.sliced.end(), i) != P.sliced.end())
        fail(MATNC_E_INVALID, "sliced ids repeat");
      P.sliced.push_back(i);
    }
    uint64_t open_mask = 0;
    for (int j = 0; j < n_open; ++j) {
      const int q = open_qubits[j];
      if (q < 0 || q >= N.n_qubits || ((open_mask >> q) & 1)) fail(MATNC_E_INVALID, "bad or repeated open qubit");
      open_mask |= 1ull << q;
    }
    P.open_qubits.assign(open_qubits, open_qubits + n_open);
    std::sort(P.open_qubits.begin(), P.open_qubits.end());
    const uint64_t valid = N.n_qubits == 64 ? ~0ull : ((1ull << N.n_qubits) - 1);
    P.words.resize((size_t)k);
    for (int64_t i = 0; i < k; ++i) {
      if (bitstrings[i] & ~valid) fail(MATNC_E_INVALID, "bitstring " + std::to_string(i) + " sets a bit >= n_qubits");
      P.words[i] = bitstrings[i] & ~open_mask;
    }
    build_structure(P);
    build_reuse(P);
    build_steps(P);
    build_memory(P);
    *out = guard.release();
  });
}

int matnc_plan_info(matnc_plan plan, matnc_plan_info_t* info) {
  return guarded([&] {
    if (!plan || !info) fail(MATNC_E_INVALID, "null argument");
    const Plan& P = plan->p;
    matnc_plan_info_t I;
    std::memset(&I, 0, sizeof(I));
    I.cmac_single = P.cmac_single;
    I.cmac_multi = P.cmac_multi;
    I.cmac_invariant = P.cmac_inv;
    I.cmac_total = P.cmac_total;
    I.bytes_per_slice = P.bytes_slice;
    I.bytes_invariant = P.bytes_inv;
    I.n_slices = (int64_t)1 << P.sliced.size();
    I.n_amplitudes = (int64_t)P.words.size() << P.open_qubits.size();
    I.n_unique = P.n_unique;
    I.max_rank = P.max_rank;
    I.n_nodes = P.net.n_tensors - 1;
    I.n_mfma_nodes = P.n_mfma;
    I.n_launches_per_batch = ((int)P.loop.size() + 2) * P.n_chunks;
    I.workspace_bytes = P.workspace_bytes;
    I.cache_bytes = P.cache_bytes;
    I.n_chunks = P.n_chunks;
    I.n_fan_nodes = 0;
    for (int v = P.net.n_tensors; v < P.n_nodes; ++v) I.n_fan_nodes += P.nodes[v].fan ? 1 : 0;
    I.n_half_nodes = P.n_half;
    *info = I;
  });
}

int matnc_plan_set_tensor(matnc_plan plan, int t, const double* data_c128) {
  return guarded([&] {
    if (!plan || !data_c128) fail(MATNC_E_INVALID, "null argument");
    Plan& P = plan->p;
    if (t < 0 || t >= P.net.n_tensors) fail(MATNC_E_INVALID, "tensor id out of range");
    const size_t ne = (size_t)1 << P.net.idx[t].size();
    P.net.data[t].assign(data_c128, data_c128 + 2 * ne);
    if (P.bound) {
      const PNode& L = P.nodes[t];
      fill_leaf_data(P, t, P.staging.data());
      hip_check(hipMemcpyAsync(reinterpret_cast<void*>(P.ws + L.off), P.staging.data() + L.off, L.buf_bytes,
                               hipMemcpyHostToDevice, P.stream),
                "upload tensor");
      if (P.precision == MATNC_CHALF) {
        const uint64_t sb = (uint64_t)L.keys.size() * (1ull << L.sl_bits.size()) * sizeof(HalfScale);
        hip_check(hipMemcpyAsync(reinterpret_cast<void*>(P.ws + L.scale_off), P.staging.data() + L.scale_off, sb,
                                 hipMemcpyHostToDevice, P.stream),
                  "upload tensor scales");
      }
      hip_check(hipStreamSynchronize(P.stream), "upload tensor");
    }
    P.inv_valid = false;
  });
}

int matnc_plan_bind(matnc_plan plan, void* dev_workspace, size_t bytes, void* hip_stream) {
  return guarded([&] {
    if (!plan || !dev_workspace) fail(MATNC_E_INVALID, "null argument");
    Plan& P = plan->p;
    if (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign) fail(MATNC_E_INVALID, "workspace not 256-byte aligned");
    if (bytes < P.workspace_bytes)
      fail(MATNC_E_NOMEM, "workspace has " + std::to_string(bytes) + " bytes, plan needs " +
                              std::to_string(P.workspace_bytes));
    bind_plan(P, dev_workspace, bytes, hip_stream, 0, nullptr);
  });
}

int matnc_execute(matnc_plan plan, int64_t slice_begin, int64_t slice_end, double* amps_dev) {
  return guarded([&] {
    if (!plan) fail(MATNC_E_INVALID, "null plan");
    Plan& P = plan->p;
    if (!P.bound) fail(MATNC_E_STATE, "execute before bind");
    if (!amps_dev) fail(MATNC_E_INVALID, "null amplitude buffer");
    const int64_t ns = (int64_t)1 << P.sliced.size();
    if (slice_begin < 0 || slice_end < slice_begin || slice_end > ns) fail(MATNC_E_INVALID, "bad slice range");
    hipStream_t st = P.stream;
    int64_t* sig = reinterpret_cast<int64_t*>(P.ws + P.sigma_off);
    claim_arena(P);
    if (!P.inv_valid) {
      hip_check(launch_set_i64(sig, 0, st), "set sigma");
      launch_prologue(P, st);
      P.inv_valid = true;
    }
    if (slice_end == slice_begin) return;
    // full batches replay graphs captured for this amplitude buffer
    const bool full = slice_end - slice_begin >= P.batch;
    if (full && st != nullptr && (P.graph_execs.empty() || P.graph_amps != amps_dev))
      capture_batch_graphs(P, amps_dev);
    const bool graphs = !P.graph_execs.empty() && P.graph_amps == amps_dev;
    for (int c = 0; c < P.n_chunks; ++c) {
      launch_chunk_prologue(P, c, st);
      for (int64_t s0 = slice_begin; s0 < slice_end; s0 += P.batch) {
        const int nb = (int)std::min<int64_t>(P.batch, slice_end - s0);
        hip_check(launch_set_i64(sig, s0, st), "set sigma");
        if (nb == P.batch && graphs)
          hip_check(hipGraphLaunch(P.graph_execs[c], st), "graph launch");
        else
          launch_batch(P, c, nb, st, amps_dev);
      }
    }
  });
}

int matnc_execute_timed(matnc_plan plan, int64_t slice_begin, int64_t slice_end, double* amps_dev, int step,
                        double* ms_total, int64_t* launches) {
  return guarded([&] {
    if (!plan || !ms_total || !launches) fail(MATNC_E_INVALID, "null argument");
    Plan& P = plan->p;
    if (!P.bound) fail(MATNC_E_STATE, "execute before bind");
    if (!amps_dev) fail(MATNC_E_INVALID, "null amplitude buffer");
    const int64_t ns = (int64_t)1 << P.sliced.size();
    if (slice_begin < 0 || slice_end < slice_begin || slice_end > ns) fail(MATNC_E_INVALID, "bad slice range");
    const int nt = P.net.n_tensors;
    if (step < 0 || step > nt - 2) fail(MATNC_E_INVALID, "step out of range");
    StepTimer T;
    T.v = nt + step;
    hipStream_t st = P.stream;
    int64_t* sig = reinterpret_cast<int64_t*>(P.ws + P.sigma_off);
    claim_arena(P);
    if (!P.inv_valid) {
      hip_check(launch_set_i64(sig, 0, st), "set sigma");
      launch_prologue(P, st, &T);
      P.inv_valid = true;
    }
    if (slice_end > slice_begin) {
      for (int c = 0; c < P.n_chunks; ++c) {
        launch_chunk_prologue(P, c, st, &T);
        for (int64_t s0 = slice_begin; s0 < slice_end; s0 += P.batch) {
          const int nb = (int)std::min<int64_t>(P.batch, slice_end - s0);
          hip_check(launch_set_i64(sig, s0, st), "set sigma");
          launch_batch(P, c, nb, st, amps_dev, &T);
        }
      }
    }
    hip_check(hipStreamSynchronize(st), "timed execute sync");
    double total = 0.0;
    for (size_t i = 0; i + 1 < T.ev.size(); i += 2) {
      float ms = 0.f;
      hip_check(hipEventElapsedTime(&ms, T.ev[i], T.ev[i + 1]), "event time");
      total += ms;
    }
    *ms_total = total;
    *launches = (int64_t)(T.ev.size() / 2);
  });
}

int matnc_xeb(matnc_plan plan, const double* amps_dev, double* xeb_dev) {
  return guarded([&] {
    if (!plan || !amps_dev || !xeb_dev) fail(MATNC_E_INVALID, "null argument");
    Plan& P = plan->p;
    if (!P.bound) fail(MATNC_E_STATE, "xeb before bind");
    const int64_t count = (int64_t)P.words.size() << P.open_qubits.size();
    hip_check(launch_xeb(amps_dev, count, P.net.n_qubits, xeb_dev, P.stream), "xeb");
  });
}

int matnc_plan_destroy(matnc_plan plan) {
  if (plan) {
    release_graph(plan->p);
    delete plan;
  }
  return MATNC_OK;
}

int matnc_plan_autotune(matnc_plan plan, int reps, const char* cache_path) {
  return guarded([&] {
    if (!plan) fail(MATNC_E_INVALID, "null plan");
    Plan& P = plan->p;
    if (!P.bound) fail(MATNC_E_STATE, "autotune before bind");
    if (reps < 1) fail(MATNC_E_INVALID, "reps must be >= 1");
    std::map<std::string, int> cache = read_tune_cache(cache_path);
    claim_arena(P);
    hipStream_t st = P.stream;
    int64_t* sig = reinterpret_cast<int64_t*>(P.ws + P.sigma_off);
    hip_check(launch_set_i64(sig, 0, st), "set sigma");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hip_check(hipEventCreate(&e0), "event create");
    hip_check(hipEventCreate(&e1), "event create");
    struct G {
      hipEvent_t a, b;
      ~G() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
      }
    } guard{e0, e1};
    std::vector<int> order(P.prologue);
    order.insert(order.end(), P.chunked.begin(), P.chunked.end());
    for (int v : order) {
      PNode& V = P.nodes[v];
      if (V.kernel != 1) continue;
      const std::string key = tune_key(P, V, node_desc(P, v, V.dep ? P.batch : 1).n_inst);
      auto it = cache.find(key);
      const bool half = V.half_store;  // FP16-product MFMA kernels
      const int ncfg = half ? mfma_h_config_count() : mfma_config_count();
      const int mb = (int)V.M.size(), nb = (int)V.N.size(), kb = (int)V.K.size();
      // fan-out steps: the configuration's N width picks the fan table
      auto cfg_tn = [&](int c) { return half ? mfma_h_config_tn(c) : mfma_config_tn(c); };
      auto config_fits = [&](int c) {
        if (V.fan) {
          const int tn = cfg_tn(c);
          if (tn != 32 && tn != 64) return false;
          return half ? mfma_h_fan_config_fits(c, mb, nb, kb, tn) : mfma_fan_config_fits(c, mb, nb, kb, tn);
        }
        return half ? mfma_h_config_fits(c, mb, nb, kb) : mfma_config_fits(c, mb, nb, kb);
      };
      auto use = [&](int c) {
        V.cfg = c;
        if (V.fan) V.fan_tn = cfg_tn(c);
      };
      if (it != cache.end()) {
        const bool fits = config_fits(it->second);
        if (fits) {
          use(it->second);
          continue;
        }
      }
      float best = 0.f;
      int best_cfg = V.cfg;
      bool have = false;
      for (int c = 0; c < ncfg; ++c) {
        if (!config_fits(c)) continue;
        use(c);
        const NodeDesc d0 = node_desc(P, v, V.dep ? P.batch : 1);
        launch_node(P, V, d0, st);  // warm-up
        // the fastest of reps separately timed launches (robust to a slow
        // outlier launch)
        float ms = 0.f;
        for (int r = 0; r < reps; ++r) {
          hip_check(hipEventRecord(e0, st), "event record");
          launch_node(P, V, d0, st);
          hip_check(hipEventRecord(e1, st), "event record");
          hip_check(hipEventSynchronize(e1), "event sync");
          float t = 0.f;
          hip_check(hipEventElapsedTime(&t, e0, e1), "event time");
          ms = r == 0 ? t : std::min(ms, t);
        }
        if (!have || ms < best) {
          have = true;
          best = ms;
          best_cfg = c;
        }
      }
      use(best_cfg);
      cache[key] = best_cfg;
    }
    hip_check(hipStreamSynchronize(st), "autotune sync");
    write_tune_cache(cache_path, cache);
    P.inv_valid = false;
    release_graph(P);
    ++P.generation;
  });
}

int matnc_plan_reset_cache(matnc_plan plan) {
  return guarded([&] {
    if (!plan) fail(MATNC_E_INVALID, "null plan");
    plan->p.inv_valid = false;
  });
}

int matnc_plan_profile(matnc_plan plan, int64_t slice_begin, int nb, float* time_ms, int* kernel, double* cmac,
                       double* bytes) {
  return guarded([&] {
    if (!plan || !time_ms || !kernel || !cmac || !bytes) fail(MATNC_E_INVALID, "null argument");
    Plan& P = plan->p;
    if (!P.bound) fail(MATNC_E_STATE, "profile before bind");
    const int64_t ns = (int64_t)1 << P.sliced.size();
    if (nb < 1 || nb > P.batch || slice_begin < 0 || slice_begin + nb > ns) fail(MATNC_E_INVALID, "bad batch");
    const int nt = P.net.n_tensors;
    const int steps = nt - 1;
    std::vector<int> order(P.prologue);
    order.insert(order.end(), P.chunked.begin(), P.chunked.end());
    std::vector<hipEvent_t> ev(2 * order.size(), nullptr);
    struct EvGuard {
      std::vector<hipEvent_t>& e;
      ~EvGuard() {
        for (auto x : e)
          if (x) (void)hipEventDestroy(x);
      }
    } eg{ev};
    for (auto& e : ev) hip_check(hipEventCreate(&e), "event create");
    claim_arena(P);
    hipStream_t st = P.stream;
    int64_t* sig = reinterpret_cast<int64_t*>(P.ws + P.sigma_off);
    hip_check(launch_set_i64(sig, 0, st), "set sigma");
    if (P.precision == MATNC_CHALF) {
      hip_check(launch_zero(P.ws + P.inv_scale_lo, P.dep_scale_hi - P.inv_scale_lo, st), "clear scales");
    }
    for (size_t i = 0; i < order.size(); ++i) {
      const int v = order[i];
      const PNode& V = P.nodes[v];
      if (i == P.prologue.size() + P.cpro.size()) hip_check(launch_set_i64(sig, slice_begin, st), "set sigma");
      const NodeDesc d = node_desc(P, v, V.dep ? nb : 1);
      hip_check(hipEventRecord(ev[2 * i], st), "event record");
      launch_node(P, V, d, st);
      hip_check(hipEventRecord(ev[2 * i + 1], st), "event record");
    }
    hip_check(hipStreamSynchronize(st), "profile sync");
    P.inv_valid = true;
    for (int j = 0; j < steps; ++j) {
      time_ms[j] = -1.f;
      kernel[j] = 0;
      cmac[j] = 0;
      bytes[j] = 0;
    }
    for (size_t i = 0; i < order.size(); ++i) {
      const int v = order[i];
      const PNode& V = P.nodes[v];
      const int j = v - nt;
      float ms = 0.f;
      hip_check(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]), "event time");
      time_ms[j] = ms;
      kernel[j] = V.kernel == 1 ? (V.half_store ? 300 : 100) + (V.fan ? 100 : 0) + V.cfg : 0;
      const NodeDesc d = node_desc(P, v, V.dep ? nb : 1);
      const double inst = (double)d.n_inst;
      cmac[j] = inst * std::ldexp(1.0, (int)(V.M.size() + V.N.size() + V.K.size()));
      const PNode& A = P.nodes[V.swap ? V.b : V.a];
      const PNode& B = P.nodes[V.swap ? V.a : V.b];
      const double ia = (double)d.A.w_child * (d.A.dep ? nb : 1);
      const double ib = (double)d.B.w_child * (d.B.dep ? nb : 1);
      bytes[j] = (double)eb_of(P, v) * inst * std::ldexp(1.0, (int)V.idx.size()) +
                 (double)eb_of(P, V.swap ? V.b : V.a) * ia * std::ldexp(1.0, (int)A.idx.size()) +
                 (double)eb_of(P, V.swap ? V.a : V.b) * ib * std::ldexp(1.0, (int)B.idx.size());
    }
  });
}

int matnc_queue_create(int n_plans, const matnc_plan* plans, matnc_queue* out) {
  return guarded([&] {
    if (n_plans < 1 || !plans || !out) fail(MATNC_E_INVALID, "bad queue arguments");
    auto q = new matnc_queue_s();
    for (int i = 0; i < n_plans; ++i) {
      if (!plans[i]) {
        delete q;
        fail(MATNC_E_INVALID, "null plan in queue");
      }
      q->plans.push_back(plans[i]);
    }
    *out = q;
  });
}

int matnc_queue_execute(matnc_queue q, double* const* amps_dev, double* xeb_dev) {
  return guarded([&] {
    if (!q || !amps_dev || !xeb_dev) fail(MATNC_E_INVALID, "null argument");
    hipStream_t st = nullptr;
    for (size_t i = 0; i < q->plans.size(); ++i) {
      const Plan& P = q->plans[i]->p;
      if (!P.bound) fail(MATNC_E_STATE, "queue plan " + std::to_string(i) + " is not bound");
      if (i == 0) st = P.stream;
      if (P.stream != st) fail(MATNC_E_INVALID, "queue plans must share one stream");
    }
    if (st == nullptr) fail(MATNC_E_INVALID, "queue plans must be bound to a non-null stream");
    std::vector<const void*> key;
    for (size_t i = 0; i < q->plans.size(); ++i) {
      if (!amps_dev[i]) fail(MATNC_E_INVALID, "null amplitude buffer in queue");
      key.push_back(amps_dev[i]);
      key.push_back(reinterpret_cast<const void*>(q->plans[i]->p.generation));
      key.push_back(reinterpret_cast<const void*>(q->plans[i]->p.ws));
    }
    key.push_back(xeb_dev);
    if (!q->exec || key != q->key) {
      if (q->exec) (void)hipGraphExecDestroy(q->exec);
      if (q->graph) (void)hipGraphDestroy(q->graph);
      q->exec = nullptr;
      q->graph = nullptr;
      hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin queue capture");
      try {
        for (size_t i = 0; i < q->plans.size(); ++i) {
          Plan& P = q->plans[i]->p;
          launch_pass(P, 0, (int64_t)1 << P.sliced.size(), amps_dev[i], st);
          const int64_t count = (int64_t)P.words.size() << P.open_qubits.size();
          hip_check(launch_xeb(amps_dev[i], count, P.net.n_qubits, xeb_dev + i, st), "xeb");
        }
      } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(st, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      hip_check(hipStreamEndCapture(st, &q->graph), "end queue capture");
      hip_check(hipGraphInstantiate(&q->exec, q->graph, nullptr, nullptr, 0), "queue graph instantiate");
      q->key = key;
    }
    hip_check(hipGraphLaunch(q->exec, st), "queue graph launch");
    // every plan's pass recomputed its stem cache; in a shared arena only
    // the last plan's survives
    for (auto p : q->plans) {
      Plan& P = p->p;
      if (P.share) {
        P.inv_valid = false;
      } else {
        P.inv_valid = true;
      }
    }
    if (q->plans.back()->p.share) {
      Plan& L = q->plans.back()->p;
      L.share->owner = L.share_id;
      L.inv_valid = true;
    }
  });
}

int matnc_queue_workspace_bytes(matnc_queue q, size_t* out) {
  return guarded([&] {
    if (!q || !out) fail(MATNC_E_INVALID, "null argument");
    uint64_t st = 0, arena = 0;
    for (auto p : q->plans) {
      const Plan& P = p->p;
      st += align_up(P.static_bytes);
      arena = std::max<uint64_t>(arena, P.workspace_bytes - P.static_bytes);
    }
    *out = (size_t)align_up(st + arena);
  });
}

int matnc_queue_bind(matnc_queue q, void* dev_workspace, size_t bytes, void* hip_stream) {
  return guarded([&] {
    if (!q || !dev_workspace) fail(MATNC_E_INVALID, "null argument");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign) fail(MATNC_E_INVALID, "workspace not 256-byte aligned");
    size_t need = 0;
    if (matnc_queue_workspace_bytes(q, &need) != MATNC_OK) fail(MATNC_E_INVALID, g_err);
    if (bytes < need)
      fail(MATNC_E_NOMEM, "workspace has " + std::to_string(bytes) + " bytes, queue needs " + std::to_string(need));
    for (size_t i = 0; i < q->plans.size(); ++i)
      for (size_t j = 0; j < i; ++j)
        if (q->plans[i] == q->plans[j]) fail(MATNC_E_INVALID, "a plan occurs twice in the queue");
    // static regions side by side, then one arena shared by all plans
    uint64_t total_static = 0;
    for (auto p : q->plans) total_static += align_up(p->p.static_bytes);
    auto share = std::make_shared<ArenaShare>();
    uint64_t prefix = 0;
    for (auto p : q->plans) {
      Plan& P = p->p;
      const uint64_t delta = total_static - prefix - P.static_bytes;
      bind_plan(P, static_cast<unsigned char*>(dev_workspace) + prefix, bytes - prefix, hip_stream, delta, share);
      prefix += align_up(P.static_bytes);
    }
    if (q->exec) (void)hipGraphExecDestroy(q->exec);
    if (q->graph) (void)hipGraphDestroy(q->graph);
    q->exec = nullptr;
    q->graph = nullptr;
    q->key.clear();
  });
}

int matnc_queue_destroy(matnc_queue q) {
  if (q) {
    if (q->exec) (void)hipGraphExecDestroy(q->exec);
    if (q->graph) (void)hipGraphDestroy(q->graph);
    delete q;
  }
  return MATNC_OK;
}

size_t matnc_contract_scratch_bytes(void) { return kContractScratchBytes; }

int matnc_mfma_config_count(void) { return mfma_config_count(); }

int matnc_contract(const void* A, const void* B, void* C, int64_t batch, int nm, int nn, int nk, const int* posA_m,
                   const int* posA_k, const int* posB_k, const int* posB_n, const int* posC_m, const int* posC_n,
                   int kernel, void* dev_scratch, size_t scratch_bytes, void* hip_stream) {
  return guarded([&] {
    if (!A || !B || !C || !dev_scratch) fail(MATNC_E_INVALID, "null argument");
    if (reinterpret_cast<uintptr_t>(dev_scratch) % kAlign) fail(MATNC_E_INVALID, "scratch not 256-byte aligned");
    if (scratch_bytes < matnc_contract_scratch_bytes()) fail(MATNC_E_NOMEM, "scratch too small");
    const ContractCall c = contract_call(batch, nm, nn, nk, posA_m, posA_k, posB_k, posB_n, posC_m, posC_n, kernel);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    // host image of the scratch: zero head (sigma slot, one zero gather
    // entry), then the six offset tables
    std::vector<unsigned char> img(matnc_contract_scratch_bytes(), 0);
    uint32_t* T = reinterpret_cast<uint32_t*>(img.data() + kAlign);
    for (int t = 0; t < TAB_COUNT; ++t)
      for (int L = 0; L < kTabLevels; ++L)
        for (int e = 0; e < kTabEntries; ++e) {
          uint32_t off = 0;
          for (int b = 0; b < 8; ++b) {
            const int bit = 8 * L + b;
            if (((e >> b) & 1) && bit < c.pos.nbits[t]) off += 1u << c.pos.pos[t][bit];
          }
          T[t * kTabSize + L * kTabEntries + e] = off;
        }
    hip_check(hipMemcpyAsync(dev_scratch, img.data(), img.size(), hipMemcpyHostToDevice, st), "upload tables");
    hip_check(hipStreamSynchronize(st), "upload tables");
    launch_contract(c, A, B, C, reinterpret_cast<uint64_t>(dev_scratch), st);
  });
}

int matnc_contract_noalloc(const void* A, const void* B, void* C, int64_t batch, int nm, int nn, int nk,
                           const int* posA_m, const int* posA_k, const int* posB_k, const int* posB_n,
                           const int* posC_m, const int* posC_n, int kernel, void* hip_stream) {
  return guarded([&] {
    if (!A || !B || !C) fail(MATNC_E_INVALID, "null argument");
    const ContractCall c = contract_call(batch, nm, nn, nk, posA_m, posA_k, posB_k, posB_n, posC_m, posC_n, kernel);
    static_assert(kContractScratchBytes <= sizeof(scratch), "static scratch smaller than one call's tables");
    const uint64_t base = reinterpret_cast<uint64_t>(static_scratch_ptr());
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    // the same scratch image as matnc_contract uploads, written by a kernel
    // on the caller's stream: no copy, no wait, nothing allocated
    hipLaunchKernelGGL(k_contract_tables, dim3(TAB_COUNT), dim3(kTabEntries), 0, st, c.pos,
                       reinterpret_cast<uint32_t*>(base));
    hip_check(hipGetLastError(), "table kernel launch");
    launch_contract(c, A, B, C, base, st);
  });
}

}  // extern "C"
