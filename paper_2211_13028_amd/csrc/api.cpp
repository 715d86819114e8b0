// Host side of rtucker: argument validation, workspace planning and the
// orchestration of the HIP kernels behind the C ABI declared in rtucker.h.
//
// Every entry point is implemented once as a "plan" that walks the same steps
// in two modes: dry (only sizes workspace by bump-allocating from address 0)
// and live (allocates from the caller's workspace and enqueues kernels).  The
// *_workspace queries run the dry mode, so the size they report is exactly
// what the live call consumes.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"

using namespace rt;

namespace {

// ------------------------------------------------------------------ context
// phases of one decomposition, as reported by rtucker_decompose_phases
enum { kPhaseSketch = 0, kPhaseQR = 1, kPhaseCore = 2, kPhaseTruncate = 3, kPhases = 4, kPhaseEnd = -1 };

struct Ctx {
  bool dry;          // size workspace only, launch nothing
  bool check_ptrs;   // validate data pointers (compute calls)
  char* base;
  size_t off = 0;
  size_t cap;
  hipStream_t st;
  hipError_t err = hipSuccess;
  size_t peak = 0;
  std::vector<PrepTask> pending;  // operand roundings not yet launched (one batched launch)
  // phase timing (rtucker_decompose_phases): an event at each phase boundary
  std::vector<hipEvent_t>* marks = nullptr;
  std::vector<int>* mark_phase = nullptr;
  void mark(int phase) {
    flush();
    if (dry || !marks) return;
    hipEvent_t e = nullptr;
    chk(hipEventCreate(&e));
    if (!e) return;
    chk(hipEventRecord(e, st));
    marks->push_back(e);
    mark_phase->push_back(phase);
  }
  void flush() {
    if (!pending.empty()) {
      if (!dry) chk(launch_prep_batch(pending.data(), static_cast<int>(pending.size()), st));
      pending.clear();
    }
  }
  void* take(size_t bytes) {
    if (bytes == 0) return nullptr;
    const size_t o = align256(off);
    off = o + align256(bytes);
    return dry ? nullptr : base + o;
  }
  void chk(hipError_t e) {
    if (err == hipSuccess && e != hipSuccess) err = e;
  }
};

struct Ten {
  std::vector<int64_t> dims;
  const void* p;
  rt_dtype dt;
  int64_t numel() const {
    int64_t n = 1;
    for (int64_t v : dims) n *= v;
    return n;
  }
  int64_t before(int k) const {
    int64_t n = 1;
    for (int i = 0; i < k; ++i) n *= dims[i];
    return n;
  }
  int64_t after(int k) const {
    int64_t n = 1;
    for (size_t i = k + 1; i < dims.size(); ++i) n *= dims[i];
    return n;
  }
};

rt_dtype ctype(rt_dtype x) { return x == RT_F64 ? RT_F64 : RT_F32; }

bool valid_dtype(int dt) { return dt >= RT_F64 && dt <= RT_F8E4M3; }

int check_tensor(const rt_tensor* X, bool need_data) {
  if (!X) return RT_EINVAL;
  if (X->d < 2 || X->d > RT_MAX_D) return RT_ESHAPE;
  for (int i = 0; i < X->d; ++i)
    if (X->dims[i] < 1) return RT_ESHAPE;
  if (!valid_dtype(X->dtype)) return RT_EDTYPE;
  if (need_data && !X->data) return RT_EINVAL;
  return RT_OK;
}

// elementwise entry points: any order 1..8, empty dimensions allowed
int check_flat(const rt_tensor* X, int64_t* n) {
  if (!X) return RT_EINVAL;
  if (X->d < 1 || X->d > RT_MAX_D) return RT_ESHAPE;
  int64_t cnt = 1;
  for (int i = 0; i < X->d; ++i) {
    if (X->dims[i] < 0) return RT_ESHAPE;
    cnt *= X->dims[i];
  }
  if (X->dtype != RT_F32 && X->dtype != RT_F64) return RT_EDTYPE;
  if (cnt > 0 && !X->data) return RT_EINVAL;
  *n = cnt;
  return RT_OK;
}

Ten ten_of(const rt_tensor* X) {
  Ten t;
  t.dims.assign(X->dims, X->dims + X->d);
  t.p = X->data;
  t.dt = X->dtype;
  return t;
}

int check_ws(const Ctx& c, void* ws, size_t ws_bytes) {
  if (c.off == 0) return RT_OK;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return RT_EWORKSPACE;
  if (ws_bytes < c.off) return RT_EWORKSPACE;
  return RT_OK;
}

// ------------------------------------------------------------------ building blocks
void* prep(Ctx& c, const double* src, int64_t m, int64_t K, bool trans, rt_dtype round_to, rt_dtype store,
           int64_t m_pad = 0) {
  if (m_pad < m) m_pad = m;
  void* dst = c.take(static_cast<size_t>(m_pad) * K * dtype_size(store));
  if (!c.dry) c.pending.push_back(PrepTask{src, m, K, m_pad, trans, round_to, store, dst});
  return dst;
}

// T x_k M, M: m x dims[k] row-major (or dims[k] x m with mtrans) in the compute type of T
Ten ttm(Ctx& c, const Ten& T, int k, const void* M, int64_t m, void* dst = nullptr, bool mtrans = false) {
  Ten out;
  out.dims = T.dims;
  out.dims[k] = m;
  out.dt = ctype(T.dt);
  const int64_t A = T.before(k), K = T.dims[k], B = T.after(k);
  void* y = dst ? dst : c.take(static_cast<size_t>(A) * m * B * dtype_size(out.dt));
  out.p = y;
  void* w = c.take(ttm_generic_ws(T.dt, A, K, B, m));
  c.flush();
  if (!c.dry) c.chk(launch_ttm_generic(T.p, T.dt, A, K, B, M, m, y, w, c.st, mtrans));
  return out;
}

struct SketchOut {
  Ten Y;              // tensor layout, compute type
  int64_t A, m, B;    // unfolding view of mode n
};

// Y_n = X x_{k != n} Phi_k for n in mask (dimension tree: one pass over X).
void sketch_impl(Ctx& c, const Ten& X, const double* const* phi, const int64_t* s, uint32_t mask,
                 std::vector<SketchOut>& out) {
  const int d = static_cast<int>(X.dims.size());
  const rt_dtype ct = ctype(X.dt);
  std::vector<const void*> op(d, nullptr);
  for (int k = 0; k < d; ++k) {
    bool need = false;
    for (int n = 0; n < d; ++n)
      if ((mask >> n & 1u) && n != k) need = true;
    if (need) op[k] = prep(c, phi ? phi[k] : nullptr, s[k], X.dims[k], false, X.dt, ct);
  }
  // tree: Z = X x_L Phi_L serves only mode S; W = X x_S Phi_S serves every other mode
  // (W is the smaller node whenever s_S I_L <= I_S s_L, and its first contraction
  // for modes n < S is over its contiguous last mode)
  const int L = d - 1, S = d - 2;
  bool needZ = false, needW = false;
  for (int n = 0; n < d; ++n)
    if (mask >> n & 1u) {
      if (n == S) needZ = true; else needW = true;
    }
  Ten Z, W;
  Z.dims = X.dims; Z.dims[L] = s[L]; Z.dt = ct; Z.p = nullptr;
  W.dims = X.dims; W.dims[S] = s[S]; W.dt = ct; W.p = nullptr;
  const int64_t A0 = X.before(S), P = X.dims[S], Q = X.dims[L];
  // the small contractions of the tree run on matrix cores when the node is binary32;
  // their padded operands are rounded now, in the same batched launch as the sketch's
  std::vector<const void*> opm(d, nullptr);
  const auto tree_kind = [&](const std::vector<int64_t>& dims, int k, bool& mf, bool& last) {
    int64_t Ab = 1, Bb = 1;
    for (int i = 0; i < k; ++i) Ab *= dims[i];
    for (int i = k + 1; i < d; ++i) Bb *= dims[i];
    mf = ct == RT_F32 && ttm_mfma_ok(RT_F32, Ab, dims[k], Bb, s[k]);
    last = ct == RT_F32 && !mf && Bb == 1 && ttm_mfma_last_ok(Ab, dims[k], s[k]);
  };
  // Memoised dimension tree below the two first-level nodes (Sec. 4.4): a node serves a
  // set M of requested modes; every mode that is neither contracted yet nor in M is
  // contracted at the node (last mode first), then M is split into halves, each served
  // by its own child.  chains[n] lists the contractions from Z (n = S) or W to Y_n;
  // targets whose chains share a prefix share the intermediate tensors of that prefix.
  std::vector<std::vector<int>> chains(d);
  std::function<void(std::vector<int>, std::vector<bool>, std::vector<int>)> assign =
      [&](std::vector<int> M, std::vector<bool> done, std::vector<int> prefix) {
        for (int k = d - 1; k >= 0; --k)
          if (!done[k] && std::find(M.begin(), M.end(), k) == M.end()) {
            prefix.push_back(k);
            done[k] = true;
          }
        if (M.size() == 1) {
          chains[M[0]] = prefix;
          return;
        }
        const size_t half = (M.size() + 1) / 2;
        assign(std::vector<int>(M.begin(), M.begin() + half), done, prefix);
        assign(std::vector<int>(M.begin() + half, M.end()), done, prefix);
      };
  {
    std::vector<int> MW;
    for (int n = 0; n < d; ++n)
      if ((mask >> n & 1u) && n != S) MW.push_back(n);
    std::vector<bool> doneW(d, false), doneZ(d, false);
    doneW[S] = true;
    doneZ[L] = true;
    if (!MW.empty()) assign(MW, doneW, {});
    if (mask >> S & 1u) assign({S}, doneZ, {});
  }
  const auto chain_of = [&](int n) { return chains[n]; };
  for (int n = 0; n < d; ++n) {
    if (!(mask >> n & 1u)) continue;
    std::vector<int64_t> dims = (n == S) ? Z.dims : W.dims;
    for (int k : chain_of(n)) {
      bool mf = false, last = false;
      tree_kind(dims, k, mf, last);
      if ((mf || last) && !opm[k])
        opm[k] = prep(c, phi ? phi[k] : nullptr, s[k], dims[k], false, X.dt, RT_F32, ttm_mfma_mpad(s[k]));
      dims[k] = s[k];
    }
  }
  if (sketch_zw_ok(X.dt, s[S], s[L])) {
    const ZWPlan plan = sketch_zw_plan(X.dt, A0, P, Q, s[S], s[L], needZ, needW);
    if (needZ) Z.p = c.take(static_cast<size_t>(Z.numel()) * dtype_size(ct));
    if (needW) W.p = c.take(static_cast<size_t>(W.numel()) * dtype_size(ct));
    void* zws = plan.ws_bytes ? c.take(plan.ws_bytes) : nullptr;
    const void* p16 = nullptr;
    const void* q16 = nullptr;
    if (plan.mfma) {  // factors rounded to X's dtype (bfloat16 storage unless binary32), padded to 16 rows
      const rt_dtype st16 = (X.dt == RT_F32) ? RT_F32 : RT_BF16;
      if (needW) p16 = prep(c, phi ? phi[S] : nullptr, s[S], P, false, X.dt, st16, 16);
      if (needZ) q16 = prep(c, phi ? phi[L] : nullptr, s[L], Q, false, X.dt, st16, 16);
    }
    c.flush();
    if (!c.dry)
      c.chk(launch_sketch_zw(X.p, X.dt, A0, P, Q, needW ? op[S] : nullptr, s[S], needZ ? op[L] : nullptr, s[L],
                             p16, q16, const_cast<void*>(Z.p), const_cast<void*>(W.p), plan, zws, c.st));
  } else {
    if (needZ) Z = ttm(c, X, L, op[L], s[L]);
    if (needW) W = ttm(c, X, S, op[S], s[S]);
  }
  // second and later levels of the tree: one tensor per distinct chain prefix; the
  // contractions of one level are independent, so the binary32 matrix-core ones go out
  // as one grouped launch
  typedef std::pair<int, std::vector<int>> NodeKey;  // (0: from Z, 1: from W; prefix)
  std::map<NodeKey, Ten> node;
  node[NodeKey{0, {}}] = Z;
  node[NodeKey{1, {}}] = W;
  size_t levels = 0;
  for (int n = 0; n < d; ++n)
    if (mask >> n & 1u) levels = std::max(levels, chains[n].size());
  for (size_t lev = 0; lev < levels; ++lev) {
    // the distinct nodes of this level, in order of their first target
    std::vector<NodeKey> keys;
    for (int n = 0; n < d; ++n) {
      if (!(mask >> n & 1u) || chains[n].size() <= lev) continue;
      NodeKey key{n == S ? 0 : 1, std::vector<int>(chains[n].begin(), chains[n].begin() + lev + 1)};
      if (std::find(keys.begin(), keys.end(), key) == keys.end()) keys.push_back(key);
    }
    std::vector<F32Contraction> group;
    std::vector<NodeKey> generic_keys, last_keys;
    std::vector<void*> last_ws;
    for (const NodeKey& key : keys) {
      const int k = key.second.back();
      const Ten& t = node.at(NodeKey{key.first, std::vector<int>(key.second.begin(), key.second.end() - 1)});
      const int64_t Ab = t.before(k), K = t.dims[k], Bb = t.after(k), m = s[k];
      bool mf = false, last = false;
      tree_kind(t.dims, k, mf, last);
      if (!mf && !last) {
        generic_keys.push_back(key);
        continue;
      }
      if (!opm[k]) opm[k] = prep(c, phi ? phi[k] : nullptr, m, K, false, X.dt, RT_F32, ttm_mfma_mpad(m));
      Ten o;
      o.dims = t.dims;
      o.dims[k] = m;
      o.dt = RT_F32;
      o.p = c.take(static_cast<size_t>(Ab) * m * Bb * sizeof(float));
      void* w = c.take(last ? ttm_mfma_last_ws(Ab, K, m) : ttm_mfma_ws(RT_F32, Ab, K, Bb, m));
      node[key] = o;
      if (last) {
        last_keys.push_back(key);
        last_ws.push_back(w);
      } else {
        group.push_back(F32Contraction{static_cast<const float*>(t.p), Ab, K, Bb, static_cast<const float*>(opm[k]), m,
                                       static_cast<float*>(const_cast<void*>(o.p)), w});
      }
    }
    c.flush();
    if (!c.dry) {
      for (size_t i = 0; i < last_keys.size(); ++i) {
        const NodeKey& key = last_keys[i];
        const int k = key.second.back();
        const Ten& t = node.at(NodeKey{key.first, std::vector<int>(key.second.begin(), key.second.end() - 1)});
        c.chk(launch_ttm_mfma_last(static_cast<const float*>(t.p), t.before(k), t.dims[k],
                                   static_cast<const float*>(opm[k]), s[k],
                                   static_cast<float*>(const_cast<void*>(node.at(key).p)), last_ws[i], c.st));
      }
      c.chk(launch_ttm_mfma_f32_group(group.data(), static_cast<int>(group.size()), c.st));
    }
    for (const NodeKey& key : generic_keys) {
      const int k = key.second.back();
      const Ten t = node.at(NodeKey{key.first, std::vector<int>(key.second.begin(), key.second.end() - 1)});
      node[key] = ttm(c, t, k, op[k], s[k]);
    }
  }
  std::vector<Ten> cur(d);
  for (int n = 0; n < d; ++n)
    if (mask >> n & 1u) cur[n] = node.at(NodeKey{n == S ? 0 : 1, chains[n]});
  out.assign(d, SketchOut{});
  for (int n = 0; n < d; ++n) {
    if (!(mask >> n & 1u)) continue;
    SketchOut o;
    o.Y = cur[n];
    o.A = cur[n].before(n);
    o.m = cur[n].dims[n];
    o.B = cur[n].after(n);
    out[n] = o;
  }
}

// G = T x_k U_k^T over the modes of mask, largest first; U_k: I_k x l_k binary64.
// With f64_out, a last contraction on the matrix-core last-mode kernel writes the core as
// binary64 directly (the same values the separate widening would give).
Ten core_impl(Ctx& c, const Ten& X, const double* const* U, const int64_t* l, uint32_t mask, void* dst,
              bool f64_out = false) {
  const int d = static_cast<int>(X.dims.size());
  std::vector<int> order;
  for (int k = 0; k < d; ++k)
    if (mask >> k & 1u) order.push_back(k);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return X.dims[a] > X.dims[b]; });
  // plan every contraction first so that all operand roundings go out in one launch
  struct Step { int k; int64_t A, K, B, m; rt_dtype in_dt; bool mfma, last, wide; const void* op; void* y; void* w; };
  std::vector<Step> steps;
  std::vector<int64_t> dims = X.dims;
  rt_dtype cur_dt = X.dt;
  for (size_t idx = 0; idx < order.size(); ++idx) {
    const int k = order[idx];
    const bool last = idx + 1 == order.size();
    Step st;
    st.k = k;
    st.A = 1; for (int i = 0; i < k; ++i) st.A *= dims[i];
    st.B = 1; for (int i = k + 1; i < d; ++i) st.B *= dims[i];
    st.K = dims[k];
    st.m = l[k];
    st.in_dt = cur_dt;
    const rt_dtype ct = ctype(cur_dt);
    st.mfma = (cur_dt == RT_F32 || cur_dt == RT_BF16) && ttm_mfma_ok(cur_dt, st.A, st.K, st.B, st.m);
    // a binary32 contraction over the last mode (B = 1) runs on the matrix-core kernel
    // for contiguous rows
    st.last = !st.mfma && cur_dt == RT_F32 && st.B == 1 && ttm_mfma_last_ok(st.A, st.K, st.m);
    st.wide = last && f64_out && st.last && !dst;
    st.y = (last && dst) ? dst
                         : c.take(static_cast<size_t>(st.A) * st.m * st.B * (st.wide ? sizeof(double) : dtype_size(ct)));
    if (st.mfma) {
      st.op = prep(c, U ? U[k] : nullptr, st.m, st.K, true, cur_dt, cur_dt, ttm_mfma_mpad(st.m));
      st.w = c.take(ttm_mfma_ws(cur_dt, st.A, st.K, st.B, st.m));
    } else if (st.last) {
      st.op = prep(c, U ? U[k] : nullptr, st.m, st.K, true, RT_F32, RT_F32, ttm_mfma_mpad(st.m));
      st.w = c.take(ttm_mfma_last_ws(st.A, st.K, st.m, st.wide));
    } else {
      st.op = prep(c, U ? U[k] : nullptr, st.m, st.K, true, cur_dt == RT_F64 ? RT_F64 : cur_dt, ct);
      st.w = c.take(ttm_generic_ws(cur_dt, st.A, st.K, st.B, st.m));
    }
    steps.push_back(st);
    dims[k] = st.m;
    cur_dt = ct;
  }
  c.flush();
  Ten cur = X;
  for (const Step& st : steps) {
    if (!c.dry) {
      if (st.mfma)
        c.chk(launch_ttm_mfma_ws(cur.p, cur.dt, st.A, st.K, st.B, st.op, st.m, static_cast<float*>(st.y), st.w, c.st));
      else if (st.last)
        c.chk(launch_ttm_mfma_last(static_cast<const float*>(cur.p), st.A, st.K, static_cast<const float*>(st.op), st.m,
                                   st.wide ? nullptr : static_cast<float*>(st.y), st.w, c.st,
                                   st.wide ? static_cast<double*>(st.y) : nullptr));
      else
        c.chk(launch_ttm_generic(cur.p, cur.dt, st.A, st.K, st.B, st.op, st.m, st.y, st.w, c.st));
    }
    Ten out;
    out.dims = cur.dims;
    out.dims[st.k] = st.m;
    out.dt = st.wide ? RT_F64 : ctype(cur.dt);
    out.p = st.y;
    cur = out;
  }
  return cur;
}

// STHOSVD of the binary64 core in mode order 1..d, then U_j = U_hat_j V_j.
void truncate_impl(Ctx& c, Ten G, const int32_t* r, double* const* Uhat, const std::vector<int64_t>& I,
                   double* Gout, double* const* Uout) {
  const int d = static_cast<int>(G.dims.size());
  std::vector<SmallGemmJob> ups;
  for (int j = 0; j < d; ++j) {
    const int64_t cj = G.dims[j], A = G.before(j), B = G.after(j), rj = r[j];
    double* gram = static_cast<double*>(c.take(static_cast<size_t>(cj) * cj * sizeof(double)));
    void* mcws = c.take(mode_contract_ws(RT_F64, A, cj, cj, B));
    double* V = static_cast<double*>(c.take(static_cast<size_t>(cj) * rj * sizeof(double)));
    if (!c.dry) {
      c.chk(launch_mode_contract(G.p, G.p, RT_F64, A, cj, cj, B, gram, mcws, c.st));
      c.chk(launch_sym_eig_top(gram, cj, rj, V, nullptr, c.st));
    }
    if (j == d - 1 && G.dt == RT_F64) {
      // the last mode is the fastest: G x_d V^T is the row-major product G_(rows) V, which
      // joins the factor updates' launch
      if (!c.dry)
        ups.push_back(SmallGemmJob{static_cast<const double*>(G.p), V, Gout, A, static_cast<int32_t>(cj),
                                   static_cast<int32_t>(rj)});
    } else {
      G = ttm(c, G, j, V, rj, (j == d - 1) ? Gout : nullptr, /*mtrans=*/true);
    }
    if (!c.dry)  // (a workspace query passes no factor arrays)
      ups.push_back(SmallGemmJob{Uhat[j], V, Uout[j], I[j], static_cast<int32_t>(cj), static_cast<int32_t>(rj)});
  }
  // the factor updates (and the last mode's contraction) do not feed the truncation: one
  // launch at the end
  if (!c.dry)
    for (size_t i = 0; i < ups.size(); i += kMaxSmallGemm)
      c.chk(launch_small_gemm_f64(ups.data() + i, static_cast<int>(std::min<size_t>(kMaxSmallGemm, ups.size() - i)),
                                  c.st));
}

Ten to_f64(Ctx& c, const Ten& T) {
  if (T.dt == RT_F64) return T;
  Ten o = T;
  o.dt = RT_F64;
  o.p = c.take(static_cast<size_t>(T.numel()) * sizeof(double));
  if (!c.dry) c.chk(launch_convert(T.p, T.dt, const_cast<void*>(o.p), RT_F64, T.numel(), 0, c.st));
  return o;
}

int64_t prod_except(const int64_t* s, int d, int n) {
  int64_t p = 1;
  for (int k = 0; k < d; ++k)
    if (k != n) p *= s[k];
  return p;
}

// exact integer version of the reuse-subrank formula
void reuse_subranks(int d, const int64_t* ell, int64_t* s) {
  // P = prod ell; s_i = least s with (s*ell_i)^(d-1) >= P.  Compare in long double
  // logs first, then confirm with exact integer arithmetic when it fits.
  for (int i = 0; i < d; ++i) {
    int64_t v = 1;
    for (;; ++v) {
      // compare (v*ell_i)^(d-1) >= prod_j ell_j  <=>  prod over j of ell_j / (v*ell_i) <= 1
      long double lhs = 1.0L;
      bool ge = false;
      // exact: accumulate ratios using integer arithmetic in 128 bits where possible
      __int128 left = 1, right = 1;
      bool overflow = false;
      for (int t = 0; t < d - 1; ++t) {
        left *= static_cast<__int128>(v * ell[i]);
        if (left > (static_cast<__int128>(1) << 100)) overflow = true;
      }
      for (int t = 0; t < d; ++t) {
        right *= ell[t];
        if (right > (static_cast<__int128>(1) << 100)) overflow = true;
      }
      if (!overflow) {
        ge = left >= right;
      } else {
        lhs = (d - 1) * logl(static_cast<long double>(v * ell[i]));
        long double rhs = 0.0L;
        for (int t = 0; t < d; ++t) rhs += logl(static_cast<long double>(ell[t]));
        ge = lhs >= rhs;
      }
      if (ge) break;
    }
    s[i] = v;
  }
}

void splits(int64_t n, int parts, int64_t lo, std::vector<int64_t>& cur, std::vector<std::vector<int64_t>>& out) {
  if (parts == 1) {
    if (n >= lo) {
      cur.push_back(n);
      out.push_back(cur);
      cur.pop_back();
    }
    return;
  }
  for (int64_t f = lo;; ++f) {
    int64_t pw = 1;
    bool big = false;
    for (int t = 0; t < parts; ++t) {
      pw *= f;
      if (pw > n) { big = true; break; }
    }
    if (big) break;
    if (n % f == 0) {
      cur.push_back(f);
      splits(n / f, parts - 1, f, cur, out);
      cur.pop_back();
    }
  }
}

// row of S: factors (non-increasing) of the least value >= ell with a (d-1)-factor split
std::vector<int64_t> sth_row(int64_t ell, int parts) {
  for (int64_t v = ell;; ++v) {
    std::vector<std::vector<int64_t>> all;
    std::vector<int64_t> cur;
    splits(v, parts, 2, cur, all);
    if (all.empty()) continue;
    for (auto& a : all) std::sort(a.begin(), a.end(), std::greater<int64_t>());
    std::sort(all.begin(), all.end());
    return all.front();
  }
}

int sizes_impl(int d, const int64_t* dims, const int32_t* r, int32_t p, rt_algo algo, int64_t* s) {
  if (d < 2 || d > RT_MAX_D || !dims || !r || !s) return RT_EINVAL;
  if (p < 0) return RT_EINVAL;
  std::vector<int64_t> ell(d);
  for (int i = 0; i < d; ++i) {
    if (dims[i] < 1 || r[i] < 1 || r[i] > dims[i]) return RT_ESHAPE;
    ell[i] = static_cast<int64_t>(r[i]) + p;
  }
  if (algo == RT_RHKRON) {
    reuse_subranks(d, ell.data(), s);
    for (int i = 0; i < d; ++i)
      if (s[i] > dims[i]) return RT_ESHAPE;
    return RT_OK;
  }
  if (algo != RT_RSTHKRON && algo != RT_RHKRON_NOREUSE) return RT_EINVAL;
  if (d == 2) {
    for (int j = 0; j < 2; ++j) {
      s[j * 2 + j] = 1;
      s[j * 2 + (1 - j)] = ell[j];
    }
  } else {
    for (int j = 0; j < d; ++j) {
      std::vector<int64_t> f = sth_row(ell[j], d - 1);
      int t = 0;
      for (int k = 0; k < d; ++k) s[j * d + k] = (k == j) ? 1 : f[t++];
    }
  }
  // sizes the factors act on: for rSTHKron the truncated c_k for k < j and I_k for k > j;
  // without reuse every factor acts on the untruncated X (I_k)
  std::vector<int64_t> cdim(d);
  for (int k = 0; k < d; ++k)
    cdim[k] = algo == RT_RSTHKRON ? std::min<int64_t>(dims[k], prod_except(s + k * d, d, k)) : dims[k];
  for (int j = 0; j < d; ++j)
    for (int k = 0; k < d; ++k)
      if (k != j && s[j * d + k] > (k < j ? cdim[k] : dims[k])) return RT_ESHAPE;
  return RT_OK;
}

// ------------------------------------------------------------------ plans
int plan_sketch(Ctx& c, const rt_tensor* X, const double* const* phi, const int64_t* s, uint32_t mask,
                void* const* Y) {
  int st = check_tensor(X, c.check_ptrs);
  if (st) return st;
  const int d = X->d;
  if (!s || mask == 0 || (mask >> d) != 0) return RT_EINVAL;
  for (int k = 0; k < d; ++k)
    if (s[k] < 1 || s[k] > X->dims[k]) return RT_ESHAPE;
  if (c.check_ptrs) {
    if (!phi || !Y) return RT_EINVAL;
    for (int n = 0; n < d; ++n) {
      if (!(mask >> n & 1u)) continue;
      if (!Y[n]) return RT_EINVAL;
      for (int k = 0; k < d; ++k)
        if (k != n && !phi[k]) return RT_EINVAL;
    }
  }
  Ten T = ten_of(X);
  std::vector<SketchOut> outs;
  sketch_impl(c, T, phi, s, mask, outs);
  const size_t es = dtype_size(ctype(X->dtype));
  c.flush();
  for (int n = 0; n < d; ++n) {
    if (!(mask >> n & 1u)) continue;
    if (!c.dry) c.chk(launch_unfold(outs[n].Y.p, es, outs[n].A, outs[n].m, outs[n].B, Y[n], c.st));
  }
  return RT_OK;
}

// the first level of the sketch's dimension tree alone: Z = X x_L Phi_L, W = X x_S Phi_S
int plan_sketch_pass(Ctx& c, const rt_tensor* X, const double* phiS, int64_t sS, const double* phiL, int64_t sL,
                     void* Z, void* W, bool wantZ, bool wantW) {
  int st = check_tensor(X, c.check_ptrs);
  if (st) return st;
  const int d = X->d;
  const int S = d - 2, L = d - 1;
  if (!wantZ && !wantW) return RT_EINVAL;
  if (wantW && (sS < 1 || sS > X->dims[S])) return RT_ESHAPE;
  if (wantZ && (sL < 1 || sL > X->dims[L])) return RT_ESHAPE;
  if (c.check_ptrs && ((wantZ && (!Z || !phiL)) || (wantW && (!W || !phiS)))) return RT_EINVAL;
  const Ten T = ten_of(X);
  const rt_dtype ct = ctype(X->dtype);
  const int64_t sP = wantW ? sS : 1, sQ = wantZ ? sL : 1;
  const void* opS = wantW ? prep(c, phiS, sS, X->dims[S], false, X->dtype, ct) : nullptr;
  const void* opL = wantZ ? prep(c, phiL, sL, X->dims[L], false, X->dtype, ct) : nullptr;
  if (sketch_zw_ok(X->dtype, sP, sQ)) {
    const int64_t A0 = T.before(S), P = X->dims[S], Q = X->dims[L];
    const ZWPlan plan = sketch_zw_plan(X->dtype, A0, P, Q, sP, sQ, wantZ, wantW);
    void* zws = plan.ws_bytes ? c.take(plan.ws_bytes) : nullptr;
    const void* p16 = nullptr;
    const void* q16 = nullptr;
    if (plan.mfma) {
      const rt_dtype st16 = (X->dtype == RT_F32) ? RT_F32 : RT_BF16;
      if (wantW) p16 = prep(c, phiS, sS, P, false, X->dtype, st16, 16);
      if (wantZ) q16 = prep(c, phiL, sL, Q, false, X->dtype, st16, 16);
    }
    c.flush();
    if (!c.dry)
      c.chk(launch_sketch_zw(X->data, X->dtype, A0, P, Q, opS, sP, opL, sQ, p16, q16, wantZ ? Z : nullptr,
                             wantW ? W : nullptr, plan, zws, c.st));
  } else {
    if (wantZ) ttm(c, T, L, opL, sL, Z);
    if (wantW) ttm(c, T, S, opS, sS, W);
  }
  return RT_OK;
}

int plan_core(Ctx& c, const rt_tensor* X, const double* const* U, const int64_t* l, uint32_t mask, void* G) {
  int st = check_tensor(X, c.check_ptrs);
  if (st) return st;
  if (X->dtype == RT_F8E4M3) return RT_EDTYPE;
  const int d = X->d;
  if (!l || mask == 0 || (mask >> d) != 0) return RT_EINVAL;
  for (int k = 0; k < d; ++k)
    if ((mask >> k & 1u) && (l[k] < 1 || l[k] > 64)) return RT_ESHAPE;
  if (c.check_ptrs) {
    if (!U || !G) return RT_EINVAL;
    for (int k = 0; k < d; ++k)
      if ((mask >> k & 1u) && !U[k]) return RT_EINVAL;
  }
  core_impl(c, ten_of(X), U, l, mask, G);
  return RT_OK;
}

int plan_qr(Ctx& c, int64_t m, int64_t n, const void* Y, rt_dtype ydt, double* Q, double* R) {
  if (m < 1 || n < 1) return RT_ESHAPE;
  if (n > kMaxQRCols) return RT_ESHAPE;
  if (ydt != RT_F32 && ydt != RT_F64) return RT_EDTYPE;
  if (c.check_ptrs && (!Y || !Q)) return RT_EINVAL;
  QRJob job{Y, 1, m, n, Q, R};
  void* w = c.take(qr_ws(&job, 1));
  if (!c.dry) c.chk(launch_qr(&job, 1, ydt, w, c.st));
  return RT_OK;
}

int plan_decompose(Ctx& c, const rt_tensor* X, const rt_tensor* Xs, const int32_t* r, int32_t p, const int64_t* s_in,
                   rt_algo algo, const double* const* phi, double* G, double* const* U) {
  int st = check_tensor(X, c.check_ptrs);
  if (st) return st;
  if (X->dtype == RT_F8E4M3) return RT_EDTYPE;
  const int d = X->d;
  if (!r || p < 0) return RT_EINVAL;
  if (algo != RT_RHKRON && algo != RT_RSTHKRON && algo != RT_RHKRON_NOREUSE) return RT_EINVAL;
  if (Xs) {
    if (algo != RT_RHKRON) return RT_EINVAL;
    st = check_tensor(Xs, c.check_ptrs);
    if (st) return st;
    if (Xs->d != d) return RT_ESHAPE;
    for (int k = 0; k < d; ++k)
      if (Xs->dims[k] != X->dims[k]) return RT_ESHAPE;
  }
  std::vector<int64_t> I(X->dims, X->dims + d);
  for (int k = 0; k < d; ++k)
    if (r[k] < 1 || r[k] > I[k]) return RT_ESHAPE;
  const int nS = (algo == RT_RHKRON) ? d : d * d;  // rSTHKron and no-reuse: the d x d matrix S
  std::vector<int64_t> s(nS);
  if (s_in) {
    std::copy(s_in, s_in + nS, s.begin());
    if (algo != RT_RHKRON)
      for (int j = 0; j < d; ++j) s[j * d + j] = 1;
  } else {
    st = sizes_impl(d, X->dims, r, p, algo, s.data());
    if (st) return st;
  }
  std::vector<int64_t> cdim(d);
  for (int n = 0; n < d; ++n) {
    const int64_t lt = (algo == RT_RHKRON) ? prod_except(s.data(), d, n) : prod_except(s.data() + n * d, d, n);
    if (lt < r[n] + static_cast<int64_t>(p)) return RT_ESHAPE;
    cdim[n] = std::min<int64_t>(I[n], lt);
    if (cdim[n] > 64) return RT_ESHAPE;
  }
  if (algo == RT_RHKRON) {
    for (int k = 0; k < d; ++k)
      if (s[k] < 1 || s[k] > I[k]) return RT_ESHAPE;
  } else {
    for (int j = 0; j < d; ++j)
      for (int k = 0; k < d; ++k)
        if (k != j && (s[j * d + k] < 1 || s[j * d + k] > ((algo == RT_RSTHKRON && k < j) ? cdim[k] : I[k])))
          return RT_ESHAPE;
  }
  if (c.check_ptrs) {
    if (!phi || !G || !U) return RT_EINVAL;
    for (int j = 0; j < d; ++j) {
      if (!U[j]) return RT_EINVAL;
      if (algo == RT_RHKRON) {
        if (!phi[j]) return RT_EINVAL;
      } else {
        for (int k = 0; k < d; ++k)
          if (k != j && !phi[j * d + k]) return RT_EINVAL;
      }
    }
  }
  std::vector<double*> Uhat(d);
  for (int n = 0; n < d; ++n) Uhat[n] = static_cast<double*>(c.take(static_cast<size_t>(I[n]) * cdim[n] * sizeof(double)));
  Ten cur = ten_of(X);
  if (algo == RT_RHKRON_NOREUSE) {
    // App. A: every mode's sketch with its own factors, each from one read of X (the
    // first level of a one-mode dimension tree), then one QR launch for all modes and the
    // core and truncation of the reuse algorithm
    std::vector<SketchOut> outs(d);
    c.mark(kPhaseSketch);
    for (int j = 0; j < d; ++j) {
      std::vector<int64_t> sj(s.begin() + j * d, s.begin() + (j + 1) * d);
      std::vector<const double*> phij(d, nullptr);
      if (phi)
        for (int k = 0; k < d; ++k) phij[k] = (k == j) ? nullptr : phi[j * d + k];
      std::vector<SketchOut> o;
      sketch_impl(c, cur, phij.data(), sj.data(), 1u << j, o);
      outs[j] = o[j];
    }
    std::vector<QRJob> jobs(d);
    for (int n = 0; n < d; ++n) jobs[n] = QRJob{outs[n].Y.p, outs[n].A, outs[n].m, outs[n].B, Uhat[n], nullptr};
    void* w = c.take(qr_ws(jobs.data(), d));
    c.mark(kPhaseQR);
    if (!c.dry) c.chk(launch_qr(jobs.data(), d, ctype(cur.dt), w, c.st));
    c.mark(kPhaseCore);
    cur = core_impl(c, cur, Uhat.data(), cdim.data(), (1u << d) - 1u, nullptr, /*f64_out=*/true);
  } else if (algo == RT_RHKRON) {
    const Ten Tsk = Xs ? ten_of(Xs) : cur;
    std::vector<SketchOut> outs;
    c.mark(kPhaseSketch);
    sketch_impl(c, Tsk, phi, s.data(), (1u << d) - 1u, outs);
    std::vector<QRJob> jobs(d);
    for (int n = 0; n < d; ++n) jobs[n] = QRJob{outs[n].Y.p, outs[n].A, outs[n].m, outs[n].B, Uhat[n], nullptr};
    void* w = c.take(qr_ws(jobs.data(), d));
    c.mark(kPhaseQR);
    if (!c.dry) c.chk(launch_qr(jobs.data(), d, ctype(Tsk.dt), w, c.st));
    c.mark(kPhaseCore);
    cur = core_impl(c, cur, Uhat.data(), cdim.data(), (1u << d) - 1u, nullptr, /*f64_out=*/true);
  } else {
    for (int j = 0; j < d; ++j) {
      std::vector<int64_t> sj(s.begin() + j * d, s.begin() + (j + 1) * d);
      std::vector<const double*> phij(d, nullptr);
      if (phi)
        for (int k = 0; k < d; ++k) phij[k] = (k == j) ? nullptr : phi[j * d + k];
      std::vector<SketchOut> outs;
      c.mark(kPhaseSketch);
      sketch_impl(c, cur, phij.data(), sj.data(), 1u << j, outs);
      QRJob job{outs[j].Y.p, outs[j].A, outs[j].m, outs[j].B, Uhat[j], nullptr};
      void* w = c.take(qr_ws(&job, 1));
      c.mark(kPhaseQR);
      if (!c.dry) c.chk(launch_qr(&job, 1, ctype(cur.dt), w, c.st));
      c.mark(kPhaseCore);
      cur = core_impl(c, cur, Uhat.data(), cdim.data(), 1u << j, nullptr, /*f64_out=*/j == d - 1);
    }
  }
  c.mark(kPhaseTruncate);
  Ten G64 = to_f64(c, cur);
  truncate_impl(c, G64, r, Uhat.data(), I, G, U);
  c.mark(kPhaseEnd);
  return RT_OK;
}

// ------------------------------------------------------------------ deterministic STHOSVD
// Alg. 2.2 on the device: for j = 1..d, the r_j leading eigenvectors V_j of the Gram matrix
// M_j of the current tensor's mode-j unfolding, then the contraction with V_j^T.  Gram
// matrices up to 64 x 64 go to the one-workgroup eigensolver; larger ones to subspace
// iteration on a block of 64 vectors, with a Rayleigh-Ritz step and a residual check every
// few iterations (the host reads one number per check), until
// max_i ||M v_i - theta_i v_i|| <= 1e-12 theta_1.
constexpr int kSubBlock = 64;
constexpr int kSubMaxIter = 400;
constexpr int kSubCheck = 4;
constexpr double kSubTol = 1e-12;

int subspace_top(Ctx& c, const double* M, int64_t n, int64_t r, double* V, int32_t* iters) {
  const int b = kSubBlock;
  double* Q = static_cast<double*>(c.take(static_cast<size_t>(n) * b * sizeof(double)));
  double* Z = static_cast<double*>(c.take(static_cast<size_t>(n) * b * sizeof(double)));
  double* H = static_cast<double*>(c.take(static_cast<size_t>(b) * b * sizeof(double)));
  double* Yv = static_cast<double*>(c.take(static_cast<size_t>(b) * r * sizeof(double)));
  double* theta = static_cast<double*>(c.take(static_cast<size_t>(r) * sizeof(double)));
  double* MV = static_cast<double*>(c.take(static_cast<size_t>(n) * r * sizeof(double)));
  double* res = static_cast<double*>(c.take(sizeof(double)));
  void* wz = c.take(ttm_generic_ws(RT_F64, 1, n, b, n));
  void* wv = c.take(ttm_generic_ws(RT_F64, 1, n, r, n));
  void* wh = c.take(mode_contract_ws(RT_F64, n, b, b, 1));
  double* T = static_cast<double*>(c.take(static_cast<size_t>(n) * b * sizeof(double)));
  QRJob job{Z, 1, n, b, Q, nullptr};
  void* wq = c.take(orth_ws(n, b));
  c.flush();
  if (c.dry) return RT_OK;
  c.chk(launch_subspace_start(Z, n, b, c.st));
  c.chk(launch_qr(&job, 1, RT_F64, wq, c.st));
  const SmallGemmJob ritz{Q, Yv, V, n, b, static_cast<int32_t>(r)};
  int it = 0;
  bool done = false;
  while (!done && c.err == hipSuccess) {
    c.chk(launch_ttm_generic(Q, RT_F64, 1, n, b, M, n, Z, wz, c.st));  // Z = M Q
    ++it;
    if (it % kSubCheck == 0 || it >= kSubMaxIter) {
      // Rayleigh-Ritz on span(Q): H = Q^T M Q, its r leading eigenpairs, V = Q Y
      c.chk(launch_mode_contract(Q, Z, RT_F64, n, b, b, 1, H, wh, c.st));
      c.chk(launch_sym_eig_top(H, b, r, Yv, theta, c.st));
      c.chk(launch_small_gemm_f64(&ritz, 1, c.st));
      c.chk(launch_ttm_generic(V, RT_F64, 1, n, r, M, n, MV, wv, c.st));
      c.chk(launch_ritz_residual(MV, V, theta, n, static_cast<int>(r), res, c.st));
      double h = 1.0;
      c.chk(hipMemcpyAsync(&h, res, sizeof(double), hipMemcpyDeviceToHost, c.st));
      c.chk(hipStreamSynchronize(c.st));
      if (h <= kSubTol) done = true;
      else if (it >= kSubMaxIter) break;
    }
    // Q = orth(M Q): the columns of M Q are as ill-conditioned as the spectrum of M is wide
    if (!done) c.chk(launch_orth(Z, n, b, T, Q, wq, c.st));
  }
  c.chk(launch_column_sign(V, n, static_cast<int>(r), c.st));
  if (iters) *iters += it;
  return done ? RT_OK : RT_ENOTCONVERGED;
}

int plan_sthosvd(Ctx& c, const rt_tensor* X, const int32_t* r, double* G, double* const* U, int32_t* iters) {
  int st = check_tensor(X, c.check_ptrs);
  if (st) return st;
  if (X->dtype != RT_F64 && X->dtype != RT_F32) return RT_EDTYPE;
  if (!r) return RT_EINVAL;
  const int d = X->d;
  for (int j = 0; j < d; ++j)
    if (r[j] < 1 || r[j] > X->dims[j] || r[j] > (X->dims[j] <= 64 ? 64 : 32)) return RT_ESHAPE;
  if (c.check_ptrs) {
    if (!G || !U) return RT_EINVAL;
    for (int j = 0; j < d; ++j)
      if (!U[j]) return RT_EINVAL;
  }
  if (iters) *iters = 0;
  Ten cur = ten_of(X);
  int status = RT_OK;
  for (int j = 0; j < d; ++j) {
    const int64_t n = cur.dims[j], A = cur.before(j), B = cur.after(j), rj = r[j];
    double* M = static_cast<double*>(c.take(static_cast<size_t>(n) * n * sizeof(double)));
    void* mcws = c.take(cur.dt == RT_F64 ? mode_contract_ws(RT_F64, A, n, n, B) : gram_wide_ws(A, n, B));
    c.flush();
    if (!c.dry) {
      if (cur.dt == RT_F64)
        c.chk(launch_mode_contract(cur.p, cur.p, RT_F64, A, n, n, B, M, mcws, c.st));
      else  // binary32 tensor: products accumulated in binary64
        c.chk(launch_gram_wide(static_cast<const float*>(cur.p), A, n, B, M, mcws, c.st));
    }
    double* V = U ? U[j] : nullptr;
    if (n <= 64) {
      if (!c.dry) c.chk(launch_sym_eig_top(M, n, rj, V, nullptr, c.st));
    } else {
      const int sst = subspace_top(c, M, n, rj, V, iters);
      if (sst == RT_ENOTCONVERGED) status = sst;
    }
    std::vector<const double*> Us(d, nullptr);
    std::vector<int64_t> l(d, 0);
    Us[j] = V;
    l[j] = rj;
    const bool last = j == d - 1;
    cur = core_impl(c, cur, Us.data(), l.data(), 1u << j, (last && cur.dt == RT_F64) ? G : nullptr);
  }
  if (cur.dt != RT_F64 && !c.dry) {
    int64_t n = 1;
    for (int j = 0; j < d; ++j) n *= r[j];
    c.chk(launch_convert(cur.p, cur.dt, G, RT_F64, n, 0, c.st));
  }
  return status;
}

int plan_rel_error(Ctx& c, const rt_tensor* X, const double* G, const int32_t* r, const double* const* U,
                   double* out) {
  int st = check_tensor(X, c.check_ptrs);
  if (st) return st;
  if (X->dtype == RT_F8E4M3) return RT_EDTYPE;
  const int d = X->d;
  if (!r) return RT_EINVAL;
  for (int k = 0; k < d; ++k)
    if (r[k] < 1 || r[k] > 64) return RT_ESHAPE;
  if (c.check_ptrs) {
    if (!G || !U || !out) return RT_EINVAL;
    for (int k = 0; k < d; ++k)
      if (!U[k]) return RT_EINVAL;
  }
  Ten T;
  T.dims.assign(r, r + d);
  T.p = G;
  T.dt = RT_F64;
  for (int k = d - 1; k >= 1; --k) T = ttm(c, T, k, U ? U[k] : nullptr, X->dims[k]);
  const int64_t Brest = T.after(0);
  void* w = c.take(recon_residual_ws(X->dims[0], Brest));
  if (!c.dry) {
    c.chk(launch_recon_residual(X->data, X->dtype, X->dims[0], Brest, U[0], static_cast<const double*>(T.p), r[0],
                                out, w, c.st));
    int64_t ng = 1;
    for (int k = 0; k < d; ++k) ng *= r[k];
    c.chk(launch_sumsq_f64(G, ng, out + 2, c.st));
  }
  return RT_OK;
}

int plan_multi_ttm(Ctx& c, const rt_tensor* X, const void* const* A, const int64_t* m, uint32_t mask, int32_t trans,
                   void* Y) {
  int st = check_tensor(X, c.check_ptrs);
  if (st) return st;
  if (X->dtype != RT_F32 && X->dtype != RT_F64) return RT_EDTYPE;
  const int d = X->d;
  if (!m || mask == 0 || (mask >> d) != 0) return RT_EINVAL;
  for (int k = 0; k < d; ++k)
    if ((mask >> k & 1u) && (m[k] < 1 || m[k] > 256)) return RT_ESHAPE;
  if (c.check_ptrs) {
    if (!A || !Y) return RT_EINVAL;
    for (int k = 0; k < d; ++k)
      if ((mask >> k & 1u) && !A[k]) return RT_EINVAL;
  }
  const size_t es = dtype_size(X->dtype);
  std::vector<int> order;
  for (int k = 0; k < d; ++k)
    if (mask >> k & 1u) order.push_back(k);
  // contract the modes that shrink the tensor most first.  Among equal ratios a
  // shrinking step goes first on the slowest mode (the full-size read is then a
  // contraction over long contiguous rows) and an expanding step goes last on it
  // (the full-size write is then coalesced).
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const double ra = static_cast<double>(m[a]) / X->dims[a], rb = static_cast<double>(m[b]) / X->dims[b];
    if (ra != rb) return ra < rb;
    return ra <= 1.0 ? a < b : a > b;
  });
  Ten cur = ten_of(X);
  for (size_t i = 0; i < order.size(); ++i) {
    const int k = order[i];
    const void* M = A ? A[k] : nullptr;
    void* dst = (i + 1 == order.size()) ? Y : nullptr;
    const int64_t Ab = cur.before(k), K = cur.dims[k], Bb = cur.after(k);
    const bool mf = X->dtype == RT_F32 && ttm_mfma_ok(RT_F32, Ab, K, Bb, m[k]);
    const bool last = X->dtype == RT_F32 && !mf && Bb == 1 && ttm_mfma_last_ok(Ab, K, m[k]);
    if (mf || last) {
      // matrix cores: operand packed to a multiple of 16 rows, binary32 accumulation
      const int64_t mp = ttm_mfma_mpad(m[k]);
      float* op = static_cast<float*>(c.take(static_cast<size_t>(mp) * K * es));
      Ten out;
      out.dims = cur.dims;
      out.dims[k] = m[k];
      out.dt = RT_F32;
      out.p = dst ? dst : c.take(static_cast<size_t>(Ab) * m[k] * Bb * es);
      void* w = c.take(last ? ttm_mfma_last_ws(Ab, K, m[k]) : ttm_mfma_ws(RT_F32, Ab, K, Bb, m[k]));
      if (!c.dry) {
        float* y = static_cast<float*>(const_cast<void*>(out.p));
        c.chk(launch_pack_f32(static_cast<const float*>(M), m[k], K, trans != 0, mp, op, c.st));
        if (last)
          c.chk(launch_ttm_mfma_last(static_cast<const float*>(cur.p), Ab, K, op, m[k], y, w, c.st));
        else
          c.chk(launch_ttm_mfma_ws(cur.p, RT_F32, Ab, K, Bb, op, m[k], y, w, c.st));
      }
      cur = out;
    } else {
      cur = ttm(c, cur, k, M, m[k], dst, trans != 0);
    }
  }
  (void)es;
  return RT_OK;
}

int plan_mode_contract(Ctx& c, const rt_tensor* P, const rt_tensor* Q, int32_t n, bool acc, void* out) {
  int st = check_tensor(P, c.check_ptrs);
  if (st) return st;
  st = check_tensor(Q, c.check_ptrs);
  if (st) return st;
  if (P->dtype != Q->dtype || (P->dtype != RT_F32 && P->dtype != RT_F64)) return RT_EDTYPE;
  if (P->d != Q->d || n < 0 || n >= P->d) return RT_EINVAL;
  for (int k = 0; k < P->d; ++k)
    if (k != n && P->dims[k] != Q->dims[k]) return RT_ESHAPE;
  if (c.check_ptrs && !out) return RT_EINVAL;
  const Ten TP = ten_of(P);
  const int64_t A = TP.before(n), B = TP.after(n);
  void* w = c.take(mode_contract_ws(P->dtype, A, P->dims[n], Q->dims[n], B));
  if (!c.dry) c.chk(launch_mode_contract(P->data, Q->data, P->dtype, A, P->dims[n], Q->dims[n], B, out, w, c.st, acc));
  return RT_OK;
}

// ------------------------------------------------------------------ batched decomposition
// Alg. 4.4 for many independent 3-way tensors of different sizes: each phase
// runs for every tensor in one grouped launch (see kernels.hpp), ~25 launches in
// all whatever the batch size.  The job tables are built on the host and live at
// the start of the workspace; `upload` copies them there (blocking), and the
// launch-only mode uses tables already in place, so it performs no host-device
// copies and can be captured in a graph.
struct BatchTune {
  int core_mt = 16;  // row tile of the vector-ALU core contractions (8, 16 or 32)
  int spb_cap = 4;   // most slabs a wave of the sketch pass takes in turn (1, 2 or 4)
};

enum class BatchMode { kFull, kUploadOnly, kLaunchOnly };

// Job tables, packed at 256-byte boundaries.  `bound` is the size the tables can take under
// any tuning (a map whose length depends on the tuning counts at its longest), so the
// workspace, which the tables open, does not depend on the tuning.
struct TableBuf {
  std::vector<unsigned char> bytes;
  size_t bound = 0;
  template <typename T>
  size_t add(const std::vector<T>& v, size_t max_count = 0) {
    const size_t off = align256(bytes.size());
    bytes.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
    bound += align256((max_count > v.size() ? max_count : v.size()) * sizeof(T));
    return off;
  }
};

int plan_batched_impl(Ctx& c, int32_t count, const rt_batch_item* items, int32_t p, rt_dtype dtype,
                      const BatchTune& tune, BatchMode mode) {
  if (count < 1 || !items || p < 0) return RT_EINVAL;
  if (dtype != RT_F32 && dtype != RT_BF16) return RT_EDTYPE;
  if (tune.core_mt != 8 && tune.core_mt != 16 && tune.core_mt != 32) return RT_EINVAL;
  if (tune.spb_cap != 1 && tune.spb_cap != 2 && tune.spb_cap != 4) return RT_EINVAL;
  const int d = 3;
  struct It {
    int64_t I[3], s[3], c[3];
    int32_t r[3];
    int order[3];
  };
  std::vector<It> its(count);
  for (int32_t i = 0; i < count; ++i) {
    const rt_batch_item& b = items[i];
    It& t = its[i];
    for (int k = 0; k < d; ++k) {
      t.I[k] = b.dims[k];
      t.r[k] = b.r[k];
      if (t.I[k] < 1 || t.r[k] < 1 || t.r[k] > t.I[k]) return RT_ESHAPE;
    }
    if (t.I[2] > 256) return RT_ESHAPE;  // one slab row per workgroup in the sketch pass
    if (b.s[0] > 0 && b.s[1] > 0 && b.s[2] > 0) {
      for (int k = 0; k < d; ++k) t.s[k] = b.s[k];
    } else {
      const int st = sizes_impl(d, t.I, t.r, p, RT_RHKRON, t.s);
      if (st) return st;
    }
    for (int k = 0; k < d; ++k) {
      if (t.s[k] < 1 || t.s[k] > t.I[k] || t.s[k] > 8) return RT_ESHAPE;
    }
    for (int n = 0; n < d; ++n) {
      const int64_t lt = prod_except(t.s, d, n);
      if (lt < t.r[n] + static_cast<int64_t>(p) || lt > 64) return RT_ESHAPE;
      t.c[n] = std::min<int64_t>(t.I[n], lt);
      if (t.I[n] > 256) return RT_ESHAPE;
    }
    for (int k = 0; k < d; ++k) t.order[k] = k;
    std::stable_sort(t.order, t.order + d, [&](int a, int b2) { return t.I[a] > t.I[b2]; });
    if (c.check_ptrs) {
      if (!b.X || !b.G) return RT_EINVAL;
      for (int k = 0; k < d; ++k)
        if (!b.phi[k] || !b.U[k]) return RT_EINVAL;
    }
  }
  const rt_dtype ct = RT_F32;
  const size_t xs = dtype_size(dtype);
  (void)xs;
  // ---- buffers and jobs
  std::vector<PrepTask> prep_sk, prep_core;
  std::vector<GZwJob> zw[4];  // by column class 4, 8, 12, 16 (index class / 4 - 1)
  std::vector<GTtmJob> tree, core[3], gttm[3], uttm[3];
  // core contractions on the batched matrix-core kernel, by step and 16-row tiles of M
  // (index: step, B == 1, 16-row tiles of M minus one)
  std::vector<GTtmJob> cb[3][2][4];
  int64_t cb_blocks[3][2][4] = {};
  std::vector<GQrJob> qr_hh, qr_fb;
  std::vector<GCholQRJob> qr_cq[2];  // by width class: at most 32 columns, at most 64
  int max_chunks[2] = {1, 1};
  std::vector<GCopyJob> cp;
  std::vector<GGramJob> gram[3];
  std::vector<GEigJob> eig[3];
  int gram_mmax[3] = {0, 0, 0}, eig_rmax[3] = {0, 0, 0};
  int64_t max_prep_sk = 1, max_prep_core = 1, max_cp = 1;
  int64_t zw_blocks[4] = {0, 0, 0, 0}, tree_blocks = 0, core_blocks[3] = {0, 0, 0}, g_blocks[3] = {0, 0, 0},
          u_blocks[3] = {0, 0, 0};
  const int core_mt_first = tune.core_mt;
  for (int32_t i = 0; i < count; ++i) {
    const rt_batch_item& b = items[i];
    const It& t = its[i];
    const int64_t I0 = t.I[0], I1 = t.I[1], I2 = t.I[2];
    // sketch operands Phi_k rounded to the tensor's dtype, binary32 storage
    float* op[3];
    for (int k = 0; k < d; ++k) {
      op[k] = static_cast<float*>(c.take(static_cast<size_t>(t.s[k]) * t.I[k] * 4));
      prep_sk.push_back(PrepTask{b.phi[k], t.s[k], t.I[k], t.s[k], false, dtype, ct, op[k]});
      max_prep_sk = std::max<int64_t>(max_prep_sk, t.s[k] * t.I[k]);
    }
    // first sketch level: Z = X x_3 Phi_3, W = X x_2 Phi_2 (one pass over X)
    float* Z = static_cast<float*>(c.take(static_cast<size_t>(I0) * I1 * t.s[2] * 4));
    float* W = static_cast<float*>(c.take(static_cast<size_t>(I0) * t.s[1] * I2 * 4));
    // a workgroup takes 4 spb slabs (spb per wave)
    const int64_t spb = std::max<int64_t>(1, std::min<int64_t>(tune.spb_cap, I0 / 32));
    const int zc = zw_batch_class(I2) / 4 - 1;
    zw[zc].push_back(GZwJob{b.X, op[1], op[2], Z, W, I0, I1, I2, zw_blocks[zc], static_cast<int32_t>(t.s[1]),
                            static_cast<int32_t>(t.s[2]), static_cast<int32_t>(spb), 0});
    zw_blocks[zc] += ceil_div(I0, 4 * spb);
    // the three sketches: Y_1 = Z x_2 Phi_2, Y_2 = Z x_1 Phi_1, Y_3 = W x_1 Phi_1
    float* Y0 = static_cast<float*>(c.take(static_cast<size_t>(I0) * t.s[1] * t.s[2] * 4));
    float* Y1 = static_cast<float*>(c.take(static_cast<size_t>(t.s[0]) * I1 * t.s[2] * 4));
    float* Y2 = static_cast<float*>(c.take(static_cast<size_t>(t.s[0]) * t.s[1] * I2 * 4));
    auto add_tree = [&](const void* X, int64_t A, int64_t K, int64_t B, const void* M, int64_t m, void* Y) {
      GTtmJob j{X, M, Y, A, K, B, m, tree_blocks, ceil_div(A * B, kWave), ceil_div(m, 8), 0, 0};
      tree_blocks += ttm_grouped_blocks(A, B, m, 8);
      tree.push_back(j);
    };
    add_tree(Z, I0, I1, t.s[2], op[1], t.s[1], Y0);
    add_tree(Z, 1, I0, I1 * t.s[2], op[0], t.s[0], Y1);
    add_tree(W, 1, I0, t.s[1] * I2, op[0], t.s[0], Y2);
    // thin QR of each sketch unfolding -> U_hat_n (I_n x c_n, binary64)
    double* Uh[3];
    const void* Ys[3] = {Y0, Y1, Y2};
    const int64_t YA[3] = {1, t.s[0], t.s[0] * t.s[1]};
    const int64_t YB[3] = {t.s[1] * t.s[2], t.s[2], 1};
    for (int n = 0; n < d; ++n) {
      Uh[n] = static_cast<double*>(c.take(static_cast<size_t>(t.I[n]) * t.c[n] * 8));
      const int64_t ncol = YA[n] * YB[n];
      if (t.I[n] >= ncol) {
        // CholeskyQR2 (tall sketch), with the Householder kernel as its fallback
        const int64_t chunks = ceil_div(t.I[n], 64);
        double* part = static_cast<double*>(c.take(static_cast<size_t>(2 * chunks) * 64 * 64 * 8));
        double* R1 = static_cast<double*>(c.take(2 * 64 * 64 * 8));  // R1, then R1^-1
        double* R2 = static_cast<double*>(c.take(2 * 64 * 64 * 8));  // R2, then R2^-1
        double* Q1 = static_cast<double*>(c.take(static_cast<size_t>(t.I[n]) * ncol * 8));
        int32_t* flag = static_cast<int32_t*>(c.take(sizeof(int32_t)));
        const int wc = ncol <= 32 ? 0 : 1;
        qr_cq[wc].push_back(GCholQRJob{Ys[n], YA[n], t.I[n], YB[n], static_cast<int32_t>(ncol), part,
                                       static_cast<int32_t>(chunks), R1, R2, Q1, Uh[n], nullptr, flag});
        qr_fb.push_back(GQrJob{Ys[n], YA[n], t.I[n], YB[n], Uh[n], static_cast<int32_t>(ncol),
                               static_cast<int32_t>(t.c[n]), flag});
        max_chunks[wc] = std::max<int>(max_chunks[wc], static_cast<int>(chunks));
      } else {
        qr_hh.push_back(GQrJob{Ys[n], YA[n], t.I[n], YB[n], Uh[n], static_cast<int32_t>(ncol),
                               static_cast<int32_t>(t.c[n]), nullptr});
      }
    }
    // core: G_hat = X x_k U_hat_k^T, largest mode first; operands rounded to the input dtype of each step
    int64_t dims[3] = {I0, I1, I2};
    const void* cur = b.X;
    for (int stp = 0; stp < d; ++stp) {
      const int k = t.order[stp];
      const rt_dtype in_dt = (stp == 0) ? dtype : ct;
      float* cop = static_cast<float*>(c.take(static_cast<size_t>(t.c[k]) * t.I[k] * 4));
      prep_core.push_back(PrepTask{Uh[k], t.c[k], t.I[k], t.c[k], true, in_dt, ct, cop});
      max_prep_core = std::max<int64_t>(max_prep_core, t.c[k] * t.I[k]);
      int64_t A = 1, B = 1;
      for (int q = 0; q < k; ++q) A *= dims[q];
      for (int q = k + 1; q < d; ++q) B *= dims[q];
      float* y = static_cast<float*>(c.take(static_cast<size_t>(A) * t.c[k] * B * 4));
      if (ttm_batch_fits(t.I[k], B, t.c[k])) {
        // matrix-core kernel (the pass over X and the later steps), jobs grouped by path and 16-row tiles of M
        const int mc = static_cast<int>(ceil_div(t.c[k], 16)) - 1, rw = B == 1 ? 1 : 0;
        const int64_t units = ttm_batch_units(A, B);
        cb[stp][rw][mc].push_back(
            GTtmJob{cur, cop, y, A, t.I[k], B, t.c[k], cb_blocks[stp][rw][mc], units, ttm_batch_row_tiles(A, B), 0, 0});
        cb_blocks[stp][rw][mc] += ttm_batch_blocks(A, B);
      } else {
        const int mt = (stp == 0) ? core_mt_first : 16;
        core[stp].push_back(GTtmJob{cur, cop, y, A, t.I[k], B, t.c[k], core_blocks[stp], ceil_div(A * B, kWave),
                                    ceil_div(t.c[k], mt), 0, 0});
        core_blocks[stp] += ttm_grouped_blocks(A, B, t.c[k], mt);
      }
      dims[k] = t.c[k];
      cur = y;
    }
    // binary64 copy of the core for the truncation
    const int64_t ng = t.c[0] * t.c[1] * t.c[2];
    double* g64 = static_cast<double*>(c.take(static_cast<size_t>(ng) * 8));
    cp.push_back(GCopyJob{static_cast<const float*>(cur), g64, ng});
    max_cp = std::max<int64_t>(max_cp, ng);
    // truncation STHOSVD(G_hat, r) in mode order 1..3, then U_j = U_hat_j V_j
    int64_t gd[3] = {t.c[0], t.c[1], t.c[2]};
    const double* gcur = g64;
    for (int j = 0; j < d; ++j) {
      const int64_t cj = gd[j];
      int64_t A = 1, B = 1;
      for (int q = 0; q < j; ++q) A *= gd[q];
      for (int q = j + 1; q < d; ++q) B *= gd[q];
      double* M = static_cast<double*>(c.take(static_cast<size_t>(cj) * cj * 8));
      double* V = static_cast<double*>(c.take(static_cast<size_t>(cj) * t.r[j] * 8));
      gram[j].push_back(GGramJob{gcur, M, A, cj, B});
      gram_mmax[j] = std::max<int>(gram_mmax[j], static_cast<int>(cj));
      eig[j].push_back(GEigJob{M, V, static_cast<int32_t>(cj), t.r[j]});
      eig_rmax[j] = std::max<int>(eig_rmax[j], t.r[j]);
      double* gnext = (j == d - 1) ? b.G : static_cast<double*>(c.take(static_cast<size_t>(A) * t.r[j] * B * 8));
      gttm[j].push_back(GTtmJob{gcur, V, gnext, A, cj, B, t.r[j], g_blocks[j], ceil_div(A * B, kWave),
                                ceil_div(t.r[j], 16), 1, 0});
      g_blocks[j] += ttm_grouped_blocks(A, B, t.r[j], 16);
      uttm[j].push_back(GTtmJob{Uh[j], V, b.U[j], t.I[j], cj, 1, t.r[j], u_blocks[j], ceil_div(t.I[j], kWave),
                                ceil_div(t.r[j], 16), 1, 0});
      u_blocks[j] += ttm_grouped_blocks(t.I[j], 1, t.r[j], 16);
      gd[j] = t.r[j];
      gcur = gnext;
    }
  }
  // ---- tables (job arrays and workgroup -> job maps), placed after every buffer
  auto ttm_map = [](const std::vector<GTtmJob>& jobs) {
    std::vector<int32_t> m;
    for (size_t j = 0; j < jobs.size(); ++j) m.insert(m.end(), jobs[j].colblocks * jobs[j].mtiles, static_cast<int32_t>(j));
    return m;
  };
  std::vector<int32_t> zw_map[4];
  for (int q = 0; q < 4; ++q)
    for (size_t j = 0; j < zw[q].size(); ++j)
      zw_map[q].insert(zw_map[q].end(), ceil_div(zw[q][j].A, 4 * zw[q][j].spb), static_cast<int32_t>(j));
  TableBuf tb;
  size_t o_zw[4], m_zw[4], o_cb[3][2][4], m_cb[3][2][4];
  for (int q = 0; q < 4; ++q) {
    o_zw[q] = tb.add(zw[q]);
    size_t most = 0;  // one slab per wave
    for (const GZwJob& j : zw[q]) most += static_cast<size_t>(ceil_div(j.A, 4));
    m_zw[q] = tb.add(zw_map[q], most);
    for (int stp = 0; stp < 3; ++stp)
      for (int rw = 0; rw < 2; ++rw) {
        std::vector<int32_t> cmap;
        for (size_t j = 0; j < cb[stp][rw][q].size(); ++j)
          cmap.insert(cmap.end(), ttm_batch_blocks(cb[stp][rw][q][j].A, cb[stp][rw][q][j].B), static_cast<int32_t>(j));
        o_cb[stp][rw][q] = tb.add(cb[stp][rw][q]);
        m_cb[stp][rw][q] = tb.add(cmap);
      }
  }
  const size_t o_psk = tb.add(prep_sk), o_tree = tb.add(tree), o_cq0 = tb.add(qr_cq[0]), o_cq1 = tb.add(qr_cq[1]),
               o_hh = tb.add(qr_hh), o_fb = tb.add(qr_fb), o_pcore = tb.add(prep_core);
  size_t o_core[3], o_gram[3], o_eig[3], o_g[3], o_u[3];
  size_t m_core[3], m_g[3], m_u[3];
  for (int q = 0; q < 3; ++q) {
    o_core[q] = tb.add(core[q]);
    size_t most = 0;  // the first contraction's smallest row tile (8) has the most workgroups
    for (const GTtmJob& j : core[q]) most += static_cast<size_t>(j.colblocks * (q == 0 ? ceil_div(j.m, 8) : j.mtiles));
    m_core[q] = tb.add(ttm_map(core[q]), most);
  }
  const size_t o_cp = tb.add(cp);
  for (int j = 0; j < 3; ++j) {
    o_gram[j] = tb.add(gram[j]);
    o_eig[j] = tb.add(eig[j]);
    o_g[j] = tb.add(gttm[j]);
    m_g[j] = tb.add(ttm_map(gttm[j]));
    o_u[j] = tb.add(uttm[j]);
    m_u[j] = tb.add(ttm_map(uttm[j]));
  }
  const size_t m_tree = tb.add(ttm_map(tree));
  char* tables = static_cast<char*>(c.take(tb.bound));
  if (c.dry) return RT_OK;
  if (mode != BatchMode::kLaunchOnly) {
    c.chk(hipMemcpyWithStream(tables, tb.bytes.data(), tb.bytes.size(), hipMemcpyHostToDevice, c.st));
    if (mode == BatchMode::kUploadOnly) return RT_OK;
  }
  auto at = [&](size_t off) { return tables + off; };
  const hipStream_t st = c.st;
  c.chk(launch_prep_grouped(reinterpret_cast<const PrepTask*>(at(o_psk)), static_cast<int>(prep_sk.size()),
                            max_prep_sk, st));
  auto imap = [&](size_t off) { return reinterpret_cast<const int32_t*>(at(off)); };
  for (int q = 0; q < 4; ++q)
    c.chk(launch_zw_batch(reinterpret_cast<const GZwJob*>(at(o_zw[q])), imap(m_zw[q]), zw_blocks[q], 4 * (q + 1),
                          dtype, st));
  c.chk(launch_ttm_grouped(reinterpret_cast<const GTtmJob*>(at(o_tree)), imap(m_tree), static_cast<int>(tree.size()),
                           tree_blocks, RT_F32, 8, st));
  c.chk(launch_cholqr2_grouped(reinterpret_cast<const GCholQRJob*>(at(o_cq0)), static_cast<int>(qr_cq[0].size()),
                               max_chunks[0], RT_F32, st, 32));
  c.chk(launch_cholqr2_grouped(reinterpret_cast<const GCholQRJob*>(at(o_cq1)), static_cast<int>(qr_cq[1].size()),
                               max_chunks[1], RT_F32, st, 64));
  c.chk(launch_qr_grouped(reinterpret_cast<const GQrJob*>(at(o_hh)), static_cast<int>(qr_hh.size()), RT_F32, st));
  c.chk(launch_qr_grouped(reinterpret_cast<const GQrJob*>(at(o_fb)), static_cast<int>(qr_fb.size()), RT_F32, st));
  c.chk(launch_prep_grouped(reinterpret_cast<const PrepTask*>(at(o_pcore)), static_cast<int>(prep_core.size()),
                            max_prep_core, st));
  for (int stp = 0; stp < 3; ++stp) {
    for (int rw = 0; rw < 2; ++rw)
      for (int q = 0; q < 4; ++q)
        c.chk(launch_ttm_batch(reinterpret_cast<const GTtmJob*>(at(o_cb[stp][rw][q])), imap(m_cb[stp][rw][q]),
                               cb_blocks[stp][rw][q], q + 1, rw == 1, stp == 0 ? dtype : RT_F32, st));
    c.chk(launch_ttm_grouped(reinterpret_cast<const GTtmJob*>(at(o_core[stp])), imap(m_core[stp]),
                             static_cast<int>(core[stp].size()), core_blocks[stp], stp == 0 ? dtype : RT_F32,
                             stp == 0 ? core_mt_first : 16, st));
  }
  c.chk(launch_copy_f64_grouped(reinterpret_cast<const GCopyJob*>(at(o_cp)), count, max_cp, st));
  for (int j = 0; j < 3; ++j) {
    c.chk(launch_gram_grouped(reinterpret_cast<const GGramJob*>(at(o_gram[j])), count, st, gram_mmax[j]));
    c.chk(launch_eig_grouped(reinterpret_cast<const GEigJob*>(at(o_eig[j])), count, st, eig_rmax[j]));
    c.chk(launch_ttm_grouped(reinterpret_cast<const GTtmJob*>(at(o_g[j])), imap(m_g[j]), count, g_blocks[j], RT_F64,
                             16, st));
    c.chk(launch_ttm_grouped(reinterpret_cast<const GTtmJob*>(at(o_u[j])), imap(m_u[j]), count, u_blocks[j], RT_F64,
                             16, st));
  }
  return RT_OK;
}

// tuned settings per batch signature (sizes, ranks, subranks, p, dtype), process-wide
std::mutex g_tune_mu;
std::map<uint64_t, BatchTune> g_tune;

uint64_t batch_key(int32_t count, const rt_batch_item* items, int32_t p, rt_dtype dtype) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a
  auto mix = [&](int64_t v) {
    for (int b = 0; b < 8; ++b) {
      h ^= static_cast<uint64_t>(v >> (8 * b)) & 0xffu;
      h *= 1099511628211ull;
    }
  };
  mix(count);
  mix(p);
  mix(dtype);
  for (int32_t i = 0; i < count && items; ++i)
    for (int k = 0; k < 3; ++k) {
      mix(items[i].dims[k]);
      mix(items[i].r[k]);
      mix(items[i].s[k]);
    }
  return h;
}

// Tuning cache file (environment variable RTUCKER_TUNE_CACHE): one line per batch
// signature, "<key, 16 hex digits> <row tile> <slabs per wave>", appended by the autotuner
// and read when a process first plans with that path set (later lines win).  Lines that
// do not parse, or hold values the plan does not accept, are skipped.
std::string g_tune_path_loaded;

void load_tune_file_locked() {
  const char* path = std::getenv("RTUCKER_TUNE_CACHE");
  if (!path || !*path || g_tune_path_loaded == path) return;
  g_tune_path_loaded = path;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof line, f)) {
    unsigned long long key = 0;
    int mt = 0, spb = 0;
    if (std::sscanf(line, "%16llx %d %d", &key, &mt, &spb) != 3) continue;
    if ((mt != 8 && mt != 16 && mt != 32) || (spb != 1 && spb != 2 && spb != 4)) continue;
    BatchTune t;
    t.core_mt = mt;
    t.spb_cap = spb;
    g_tune[static_cast<uint64_t>(key)] = t;
  }
  std::fclose(f);
}

void save_tune_locked(uint64_t key, const BatchTune& t) {
  g_tune[key] = t;
  const char* path = std::getenv("RTUCKER_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;  // the cache is an optimisation: an unwritable path only loses it
  std::fprintf(f, "%016llx %d %d\n", static_cast<unsigned long long>(key), t.core_mt, t.spb_cap);
  std::fclose(f);
}

BatchTune tune_for(int32_t count, const rt_batch_item* items, int32_t p, rt_dtype dtype) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_tune_file_locked();
  auto it = g_tune.find(batch_key(count, items, p, dtype));
  return it == g_tune.end() ? BatchTune{} : it->second;
}

int plan_batched(Ctx& c, int32_t count, const rt_batch_item* items, int32_t p, rt_dtype dtype,
                 BatchMode mode = BatchMode::kFull) {
  return plan_batched_impl(c, count, items, p, dtype, tune_for(count, items, p, dtype), mode);
}

template <typename F>
int run(F&& plan, void* ws, size_t ws_bytes, void* stream) {
  Ctx dry{true, true, nullptr, 0, 0, nullptr};
  int st = plan(dry);
  if (st) return st;
  Ctx live{false, true, static_cast<char*>(ws), 0, ws_bytes, static_cast<hipStream_t>(stream)};
  st = check_ws(dry, ws, ws_bytes);
  if (st) return st;
  st = plan(live);
  live.flush();
  if (st) return st;
  return live.err == hipSuccess ? RT_OK : RT_EHIP;
}

// run() with an event at every phase boundary; synchronises `stream` and sums the
// intervals per phase (milliseconds) into phase_ms[kPhases]
template <typename F>
int run_timed(F&& plan, void* ws, size_t ws_bytes, void* stream, float* phase_ms) {
  Ctx dry{true, true, nullptr, 0, 0, nullptr};
  int st = plan(dry);
  if (st) return st;
  st = check_ws(dry, ws, ws_bytes);
  if (st) return st;
  std::vector<hipEvent_t> marks;
  std::vector<int> phase;
  Ctx live{false, true, static_cast<char*>(ws), 0, ws_bytes, static_cast<hipStream_t>(stream)};
  live.marks = &marks;
  live.mark_phase = &phase;
  st = plan(live);
  live.flush();
  if (st == RT_OK && live.err == hipSuccess) live.chk(hipStreamSynchronize(live.st));
  for (int k = 0; k < kPhases; ++k) phase_ms[k] = 0.f;
  for (size_t i = 0; i + 1 < marks.size(); ++i) {
    float ms = 0.f;
    if (live.err == hipSuccess) live.chk(hipEventElapsedTime(&ms, marks[i], marks[i + 1]));
    if (phase[i] >= 0 && phase[i] < kPhases) phase_ms[phase[i]] += ms;
  }
  for (hipEvent_t e : marks) hipEventDestroy(e);
  if (st) return st;
  return live.err == hipSuccess ? RT_OK : RT_EHIP;
}

template <typename F>
int query(F&& plan, size_t* bytes) {
  if (!bytes) return RT_EINVAL;
  Ctx dry{true, false, nullptr, 0, 0, nullptr};
  const int st = plan(dry);
  if (st) return st;
  *bytes = dry.off ? align256(dry.off) : 0;
  return RT_OK;
}

}  // namespace

// ------------------------------------------------------------------ static scratch
// Workspace of rtucker_decompose_noalloc: a file-scope device array, one copy per GPU
// the library runs on, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in symbol): its device
// address is looked up once per device with hipGetSymbolAddress and kept here.
constexpr size_t kScratchBytes = static_cast<size_t>(RTUCKER_NOALLOC_SCRATCH_BYTES);
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device ordinal -> address of that device's scratch

int scratch_for_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return RT_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return RT_EHIP;
    it = g_scratch_ptr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return RT_OK;
}

// ====================================================================== C ABI
extern "C" {

const char* rtucker_status_string(int status) {
  switch (status) {
    case RT_OK: return "ok";
    case RT_EINVAL: return "invalid argument";
    case RT_ESHAPE: return "inconsistent or unsupported shape";
    case RT_EDTYPE: return "unsupported dtype";
    case RT_EWORKSPACE: return "workspace missing, misaligned or too small";
    case RT_EHIP: return "HIP runtime error";
    case RT_ENOTCONVERGED: return "iterative eigensolver did not converge";
    default: return "unknown status";
  }
}

const char* rtucker_version(void) { return "rtucker 0.1 (gfx950)"; }

int rtucker_sketch_sizes(int32_t d, const int64_t* dims, const int32_t* r, int32_t p, rt_algo algo, int64_t* s_out) {
  return sizes_impl(d, dims, r, p, algo, s_out);
}

int rtucker_sketch_workspace(const rt_tensor* X, const int64_t* s, uint32_t mode_mask, size_t* bytes) {
  return query([&](Ctx& c) { return plan_sketch(c, X, nullptr, s, mode_mask, nullptr); }, bytes);
}

int rtucker_sketch(const rt_tensor* X, const double* const* phi, const int64_t* s, uint32_t mode_mask, void* const* Y,
                   void* ws, size_t ws_bytes, void* stream) {
  return run([&](Ctx& c) { return plan_sketch(c, X, phi, s, mode_mask, Y); }, ws, ws_bytes, stream);
}

int rtucker_qr_workspace(int64_t m, int64_t n, size_t* bytes) {
  return query([&](Ctx& c) { return plan_qr(c, m, n, nullptr, RT_F64, nullptr, nullptr); }, bytes);
}

int rtucker_qr(int64_t m, int64_t n, const void* Y, rt_dtype y_dtype, double* Q, double* R, void* ws, size_t ws_bytes,
               void* stream) {
  return run([&](Ctx& c) { return plan_qr(c, m, n, Y, y_dtype, Q, R); }, ws, ws_bytes, stream);
}

int rtucker_core_workspace(const rt_tensor* X, const int64_t* l, uint32_t mode_mask, size_t* bytes) {
  return query([&](Ctx& c) { return plan_core(c, X, nullptr, l, mode_mask, nullptr); }, bytes);
}

int rtucker_core(const rt_tensor* X, const double* const* U, const int64_t* l, uint32_t mode_mask, void* G, void* ws,
                 size_t ws_bytes, void* stream) {
  return run([&](Ctx& c) { return plan_core(c, X, U, l, mode_mask, G); }, ws, ws_bytes, stream);
}

int rtucker_decompose_workspace(const rt_tensor* X, const rt_tensor* X_sketch, const int32_t* r, int32_t p,
                                const int64_t* s, rt_algo algo, size_t* bytes) {
  return query([&](Ctx& c) { return plan_decompose(c, X, X_sketch, r, p, s, algo, nullptr, nullptr, nullptr); },
               bytes);
}

int rtucker_decompose(const rt_tensor* X, const rt_tensor* X_sketch, const int32_t* r, int32_t p, const int64_t* s,
                      rt_algo algo, const double* const* phi, double* G, double* const* U, void* ws, size_t ws_bytes,
                      void* stream) {
  return run([&](Ctx& c) { return plan_decompose(c, X, X_sketch, r, p, s, algo, phi, G, U); }, ws, ws_bytes, stream);
}

int rtucker_decompose_phases(const rt_tensor* X, const rt_tensor* X_sketch, const int32_t* r, int32_t p,
                             const int64_t* s, rt_algo algo, const double* const* phi, double* G, double* const* U,
                             void* ws, size_t ws_bytes, void* stream, float* phase_ms) {
  if (!phase_ms) return RT_EINVAL;
  return run_timed([&](Ctx& c) { return plan_decompose(c, X, X_sketch, r, p, s, algo, phi, G, U); }, ws, ws_bytes,
                   stream, phase_ms);
}

int rtucker_decompose_noalloc(const rt_tensor* X, const rt_tensor* X_sketch, const int32_t* r, int32_t p,
                              const int64_t* s, rt_algo algo, const double* const* phi, double* G, double* const* U,
                              void* stream) {
  size_t need = 0;
  int st = query([&](Ctx& c) { return plan_decompose(c, X, X_sketch, r, p, s, algo, nullptr, nullptr, nullptr); },
                 &need);
  if (st) return st;
  if (need > kScratchBytes) return RT_EWORKSPACE;
  void* ws = nullptr;
  st = scratch_for_current_device(&ws);
  if (st) return st;
  return run([&](Ctx& c) { return plan_decompose(c, X, X_sketch, r, p, s, algo, phi, G, U); }, ws, kScratchBytes,
             stream);
}

int rtucker_sthosvd_workspace(const rt_tensor* X, const int32_t* r, size_t* bytes) {
  return query([&](Ctx& c) { return plan_sthosvd(c, X, r, nullptr, nullptr, nullptr); }, bytes);
}

int rtucker_sthosvd(const rt_tensor* X, const int32_t* r, double* G, double* const* U, int32_t* iterations,
                    void* ws, size_t ws_bytes, void* stream) {
  const int st = run([&](Ctx& c) { return plan_sthosvd(c, X, r, G, U, c.dry ? nullptr : iterations); }, ws,
                     ws_bytes, stream);
  if (st != RT_OK) return st;
  return hipStreamSynchronize(static_cast<hipStream_t>(stream)) == hipSuccess ? RT_OK : RT_EHIP;
}

int rtucker_rel_error_workspace(const rt_tensor* X, const int32_t* r, size_t* bytes) {
  return query([&](Ctx& c) { return plan_rel_error(c, X, nullptr, r, nullptr, nullptr); }, bytes);
}

int rtucker_rel_error(const rt_tensor* X, const double* G, const int32_t* r, const double* const* U, double* out,
                      void* ws, size_t ws_bytes, void* stream) {
  return run([&](Ctx& c) { return plan_rel_error(c, X, G, r, U, out); }, ws, ws_bytes, stream);
}

int rtucker_convert(const void* src, rt_dtype src_dtype, void* dst, rt_dtype dst_dtype, int64_t n, int32_t scale_exp,
                    void* stream) {
  if (n < 0) return RT_EINVAL;
  if (src_dtype != RT_F64 && src_dtype != RT_F32) return RT_EDTYPE;
  if (dst_dtype != RT_F32 && dst_dtype != RT_BF16 && dst_dtype != RT_F8E4M3) return RT_EDTYPE;
  if (scale_exp < -1000 || scale_exp > 1000) return RT_EINVAL;
  if (n == 0) return RT_OK;
  if (!src || !dst) return RT_EINVAL;
  return launch_convert(src, src_dtype, dst, dst_dtype, n, scale_exp, static_cast<hipStream_t>(stream)) == hipSuccess
             ? RT_OK
             : RT_EHIP;
}

int rtucker_srht_factor(int64_t n, int64_t s, const int64_t* rows, const double* signs, double* phi,
                        void* stream) {
  if (n < 1 || s < 1) return RT_ESHAPE;
  int64_t N = 1;
  while (N < n) N *= 2;
  if (s > N) return RT_ESHAPE;
  if (!rows || !signs || !phi) return RT_EINVAL;
  return launch_srht_factor(n, s, rows, signs, 1.0 / std::sqrt(static_cast<double>(N)), phi,
                            static_cast<hipStream_t>(stream)) == hipSuccess
             ? RT_OK
             : RT_EHIP;
}

int rtucker_srht_sketch_last(const rt_tensor* X, int64_t s, const int64_t* rows, const double* signs, float* Z,
                             void* stream) {
  int64_t n = 0;
  const int st = check_flat(X, &n);
  if (st) return st;
  if (X->dtype != RT_F32) return RT_EDTYPE;
  const int64_t Q = X->dims[X->d - 1];
  if (!srht_last_ok(Q, s)) return RT_ESHAPE;
  if (n == 0) return RT_OK;
  if (!rows || !signs || !Z) return RT_EINVAL;
  return launch_srht_last(static_cast<const float*>(X->data), n / Q, Q, rows, signs, s, Z,
                          static_cast<hipStream_t>(stream)) == hipSuccess
             ? RT_OK
             : RT_EHIP;
}

int rtucker_multi_ttm_workspace(const rt_tensor* X, const int64_t* m, uint32_t mode_mask, size_t* bytes) {
  return query([&](Ctx& c) { return plan_multi_ttm(c, X, nullptr, m, mode_mask, 1, nullptr); }, bytes);
}

int rtucker_multi_ttm(const rt_tensor* X, const void* const* A, const int64_t* m, uint32_t mode_mask,
                      int32_t transpose, void* Y, void* ws, size_t ws_bytes, void* stream) {
  return run([&](Ctx& c) { return plan_multi_ttm(c, X, A, m, mode_mask, transpose, Y); }, ws, ws_bytes, stream);
}

int rtucker_mode_contract_workspace(const rt_tensor* P, const rt_tensor* Q, int32_t n, size_t* bytes) {
  return query([&](Ctx& c) { return plan_mode_contract(c, P, Q, n, false, nullptr); }, bytes);
}

int rtucker_mode_contract(const rt_tensor* P, const rt_tensor* Q, int32_t n, int32_t accumulate, void* out, void* ws,
                          size_t ws_bytes, void* stream) {
  return run([&](Ctx& c) { return plan_mode_contract(c, P, Q, n, accumulate != 0, out); }, ws, ws_bytes, stream);
}

int rtucker_sq_residual(const rt_tensor* A, const void* B, void* R, double* out, void* ws, size_t ws_bytes,
                        void* stream) {
  int64_t n = 0;
  const int st = check_flat(A, &n);
  if (st) return st;
  if ((n > 0 && !B) || !out) return RT_EINVAL;
  const size_t need = sq_residual_ws(n);
  if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255u)) return RT_EWORKSPACE;
  return launch_sq_residual(A->data, B, R, A->dtype, n, out, ws, static_cast<hipStream_t>(stream)) == hipSuccess
             ? RT_OK
             : RT_EHIP;
}

int rtucker_sketch_pass_workspace(const rt_tensor* X, int64_t s_prev, int64_t s_last, size_t* bytes) {
  return query([&](Ctx& c) { return plan_sketch_pass(c, X, nullptr, s_prev, nullptr, s_last, nullptr, nullptr, true, true); },
               bytes);
}

int rtucker_sketch_pass(const rt_tensor* X, const double* phi_prev, int64_t s_prev, const double* phi_last,
                        int64_t s_last, void* Z, void* W, void* ws, size_t ws_bytes, void* stream) {
  return run([&](Ctx& c) { return plan_sketch_pass(c, X, phi_prev, s_prev, phi_last, s_last, Z, W, Z != nullptr, W != nullptr); },
             ws, ws_bytes, stream);
}

int rtucker_scaled_diff(const rt_tensor* A, const void* B, const double* g, double alpha, void* out,
                        void* stream) {
  int64_t n = 0;
  const int st = check_flat(A, &n);
  if (st) return st;
  if (n > 0 && !out) return RT_EINVAL;
  return launch_scaled_diff(A->data, B, g, alpha, A->dtype, n, out, static_cast<hipStream_t>(stream)) == hipSuccess
             ? RT_OK
             : RT_EHIP;
}

int rtucker_decompose_batched_workspace(int32_t count, const rt_batch_item* items, int32_t p, rt_dtype dtype,
                                        size_t* bytes) {
  return query([&](Ctx& c) { return plan_batched(c, count, items, p, dtype); }, bytes);
}

int rtucker_decompose_batched(int32_t count, const rt_batch_item* items, int32_t p, rt_dtype dtype, void* ws,
                              size_t ws_bytes, void* stream) {
  return run([&](Ctx& c) { return plan_batched(c, count, items, p, dtype); }, ws, ws_bytes, stream);
}

int rtucker_decompose_batched_upload(int32_t count, const rt_batch_item* items, int32_t p, rt_dtype dtype, void* ws,
                                     size_t ws_bytes, void* stream) {
  return run([&](Ctx& c) { return plan_batched(c, count, items, p, dtype, BatchMode::kUploadOnly); }, ws, ws_bytes,
             stream);
}

int rtucker_decompose_batched_launch(int32_t count, const rt_batch_item* items, int32_t p, rt_dtype dtype, void* ws,
                                     size_t ws_bytes, void* stream) {
  return run([&](Ctx& c) { return plan_batched(c, count, items, p, dtype, BatchMode::kLaunchOnly); }, ws, ws_bytes,
             stream);
}

int rtucker_decompose_batched_tuning(int32_t count, const rt_batch_item* items, int32_t p, rt_dtype dtype,
                                     int32_t* tuning, uint64_t* key) {
  if (count < 1 || !items || !tuning || p < 0) return RT_EINVAL;
  if (dtype != RT_F32 && dtype != RT_BF16) return RT_EDTYPE;
  const BatchTune t = tune_for(count, items, p, dtype);
  tuning[0] = t.core_mt;
  tuning[1] = t.spb_cap;
  if (key) *key = batch_key(count, items, p, dtype);
  return RT_OK;
}

int rtucker_decompose_batched_autotune(int32_t count, const rt_batch_item* items, int32_t p, rt_dtype dtype,
                                       void* ws, size_t ws_bytes, void* stream, int32_t* chosen) {
  const int mts[3] = {8, 16, 32};
  const int spbs[3] = {1, 2, 4};
  float best_ms = -1.0f;
  BatchTune best;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return RT_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return RT_EHIP;
  }
  int status = RT_OK;
  for (int ci = 0; ci < 9 && status == RT_OK; ++ci) {
    BatchTune tune;
    tune.core_mt = mts[ci % 3];
    tune.spb_cap = spbs[ci / 3];
    auto plan = [&](Ctx& c, BatchMode m) { return plan_batched_impl(c, count, items, p, dtype, tune, m); };
    status = run([&](Ctx& c) { return plan(c, BatchMode::kUploadOnly); }, ws, ws_bytes, stream);
    if (status) break;
    status = run([&](Ctx& c) { return plan(c, BatchMode::kLaunchOnly); }, ws, ws_bytes, stream);  // warm-up
    if (status) break;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipEventRecord(e0, st) != hipSuccess) { status = RT_EHIP; break; }
    for (int rep = 0; rep < 3 && status == RT_OK; ++rep)
      status = run([&](Ctx& c) { return plan(c, BatchMode::kLaunchOnly); }, ws, ws_bytes, stream);
    if (status) break;
    float ms = 0.0f;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      status = RT_EHIP;
      break;
    }
    if (best_ms < 0.0f || ms < best_ms) {
      best_ms = ms;
      best = tune;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status) return status;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file_locked();
    save_tune_locked(batch_key(count, items, p, dtype), best);
  }
  if (chosen) {
    chosen[0] = best.core_mt;
    chosen[1] = best.spb_cap;
  }
  // leave the tables of the chosen setting in the workspace for a following launch-only call
  return run([&](Ctx& c) { return plan_batched(c, count, items, p, dtype, BatchMode::kUploadOnly); }, ws, ws_bytes,
             stream);
}

}  // extern "C"
