// C ABI and host-side plan construction of the layered-media FMM.
//
// Design (Sec. 3.3, Algorithms 1 and 2, with the polarization sources of
// eq. eqpolarizedsource): every reaction component pairs a target layer l,
// seen from one of its interfaces (a = 1: heights above d_l; a = 2: depths
// below d_{l-1}), with a source layer l' seen from one of its interfaces
// (b = 1: heights above d_l'; b = 2: depths below d_{l'-1}).  In the frame of
// the target interface the targets sit at height h_t > 0 and the polarization
// sources at -h_s, and the component depends only on rho and h_t + h_s
// (eq. zexponential).  So one octree per (layer, side) -- 2L trees, all with
// the same root side W and xy origin, each root cube resting on its interface
// -- serves as target tree and (mirrored) source tree of every component, and
// the free-space FMM of each layer runs in one of its layer's trees.  The
// centre conditions of eq. imagecentercond hold by construction, and every
// M2L offset is an integer multiple of the box size, so the reaction
// operators depend only on (component, level, offset).
//
// Interaction lists come from a dual-tree traversal of same-level box pairs:
// adjacent pairs recurse into their children, separated children are M2L
// pairs, and a pair with a leaf on either side is handled directly (P2P
// between the two subtrees).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <unordered_set>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "fmm_internal.h"

namespace fmmlm {

thread_local std::string g_last_error;
void set_last_error(const std::string& s) { g_last_error = s; }

namespace {

struct HBox {
  uint64_t prefix;
  int level;
  int tree;
  int64_t start, count;  // global tree-order point range
  int parent;            // global id
  int child0, nchild;    // global ids
  int ix, iy, ih;
};

template <class T>
int dev_alloc(fmmlm_plan_s* P, T** out, size_t count) {
  *out = nullptr;
  if (count == 0) count = 1;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, count * sizeof(T));
  if (e != hipSuccess) {
    set_last_error(std::string("hipMalloc: ") + hipGetErrorString(e));
    return FMMLM_ENOMEM;
  }
  P->bufs.push_back(DevBuf{p, count * sizeof(T)});
  P->device_bytes += (int64_t)(count * sizeof(T));
  *out = static_cast<T*>(p);
  return FMMLM_OK;
}

template <class T>
int dev_upload(fmmlm_plan_s* P, T** out, const std::vector<T>& v, hipStream_t st) {
  int rc = dev_alloc(P, out, v.size());
  if (rc) return rc;
  if (!v.empty()) FMM_HIP_TRY(hipMemcpyAsync(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return FMMLM_OK;
}

bool is_device_ptr(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice;
}

template <class T>
int fetch(const T* src, int64_t n, std::vector<T>& dst) {
  dst.resize(n);
  if (n == 0) return FMMLM_OK;
  if (is_device_ptr(src)) {
    FMM_HIP_TRY(hipMemcpy(dst.data(), src, n * sizeof(T), hipMemcpyDeviceToHost));
  } else {
    std::memcpy(dst.data(), src, n * sizeof(T));
  }
  return FMMLM_OK;
}

inline uint64_t spread1by2(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

inline int compact1by2(uint64_t v) {
  v &= 0x1249249249249249ull;
  v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
  v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
  v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
  v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
  v = (v ^ (v >> 32)) & 0x1fffffull;
  return (int)v;
}

struct Builder {
  fmmlm_plan_s* P;
  int mac_d2 = 4;
  std::vector<HBox> boxes;                 // global, level-major
  std::vector<int> root;                   // per tree
  // M2L triples
  std::vector<int> m_tgt, m_src, m_op;
  std::vector<char> m_isfree;
  // free ops by offset code
  std::vector<int> free_code_to_op;
  std::vector<int> free_off;               // 3 per op
  // reaction ops
  std::map<std::tuple<int, int, int, int, int>, int> reac_op_id;  // (comp, level, dx, dy, dz)
  std::map<std::tuple<int, int, int, int>, int> task_id;          // (comp, level, r2, dz)
  std::vector<int> reac_task;
  std::vector<double> reac_phi, reac_S;
  std::vector<SommTask> tasks;
  // P2P
  std::vector<std::vector<std::pair<int, int>>> p2p_free;   // per box (leaf) : (start, count)
  struct RP {
    int start, count, comp;
  };
  std::vector<std::vector<RP>> p2p_reac;                    // per box (leaf)
  int64_t free_pairs = 0, reac_pairs = 0;

  bool leaf(int b) const { return boxes[b].nchild == 0; }

  void leaves_of(int b, std::vector<int>& out) const {
    if (leaf(b)) {
      out.push_back(b);
      return;
    }
    for (int c = 0; c < boxes[b].nchild; ++c) leaves_of(boxes[b].child0 + c, out);
  }

  void add_p2p_free(int B, int C) {
    std::vector<int> lv;
    leaves_of(B, lv);
    for (int b : lv) {
      p2p_free[b].push_back({(int)boxes[C].start, (int)boxes[C].count});
      free_pairs += boxes[b].count * boxes[C].count;
    }
  }

  void add_p2p_reac(int B, int C, int comp) {
    std::vector<int> lv;
    leaves_of(B, lv);
    for (int b : lv) {
      p2p_reac[b].push_back({(int)boxes[C].start, (int)boxes[C].count, comp});
      reac_pairs += boxes[b].count * boxes[C].count;
    }
  }

  void process_free(int B, int C) {
    if (leaf(B) || leaf(C)) {
      add_p2p_free(B, C);
      return;
    }
    const HBox& bb = boxes[B];
    const HBox& cc = boxes[C];
    for (int i = 0; i < bb.nchild; ++i) {
      const int b = bb.child0 + i;
      for (int j = 0; j < cc.nchild; ++j) {
        const int c = cc.child0 + j;
        const int dx = boxes[b].ix - boxes[c].ix, dy = boxes[b].iy - boxes[c].iy, dz = boxes[b].ih - boxes[c].ih;
        const bool adjacent = std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1;
        if (adjacent || dx * dx + dy * dy + dz * dz < mac_d2) {
          process_free(b, c);
        } else {
          const int code = (dx + 7) * 225 + (dy + 7) * 15 + (dz + 7);
          if (free_code_to_op[code] < 0) {
            free_code_to_op[code] = (int)(free_off.size() / 3);
            free_off.push_back(dx);
            free_off.push_back(dy);
            free_off.push_back(dz);
          }
          m_tgt.push_back(b);
          m_src.push_back(c);
          m_op.push_back(free_code_to_op[code]);
          m_isfree.push_back(1);
        }
      }
    }
  }

  void process_reac(int B, int C, int comp) {
    if (leaf(B) || leaf(C)) {
      add_p2p_reac(B, C, comp);
      return;
    }
    const HBox& bb = boxes[B];
    const HBox& cc = boxes[C];
    for (int i = 0; i < bb.nchild; ++i) {
      const int b = bb.child0 + i;
      for (int j = 0; j < cc.nchild; ++j) {
        const int c = cc.child0 + j;
        const int dx = boxes[b].ix - boxes[c].ix, dy = boxes[b].iy - boxes[c].iy;
        const int dz = boxes[b].ih + boxes[c].ih + 1;  // target above, mirrored source below
        const bool adjacent = std::abs(dx) <= 1 && std::abs(dy) <= 1 && dz == 1;
        if (adjacent || dx * dx + dy * dy + dz * dz < mac_d2) {
          process_reac(b, c, comp);
        } else {
          const int lvl = boxes[b].level;
          auto key = std::make_tuple(comp, lvl, dx, dy, dz);
          auto it = reac_op_id.find(key);
          int op;
          if (it == reac_op_id.end()) {
            const int r2 = dx * dx + dy * dy;
            auto tkey = std::make_tuple(comp, lvl, r2, dz);
            auto tt = task_id.find(tkey);
            int tid;
            const double S = P->W / std::ldexp(1.0, lvl);
            if (tt == task_id.end()) {
              tid = (int)tasks.size();
              task_id[tkey] = tid;
              tasks.push_back(SommTask{comp, S, S * std::sqrt((double)r2), S * dz});
            } else {
              tid = tt->second;
            }
            op = (int)reac_task.size();
            reac_op_id[key] = op;
            reac_task.push_back(tid);
            reac_phi.push_back(std::atan2((double)dy, (double)dx));
            reac_S.push_back(S);
          } else {
            op = it->second;
          }
          m_tgt.push_back(b);
          m_src.push_back(c);
          m_op.push_back(op);
          m_isfree.push_back(0);
        }
      }
    }
  }
};

// Largest deviation of the learned or table form from the quadrature on a
// plan's sampled tasks (interaction units, fmmlm_stats.surrogate_check) that the
// plan accepts; above it the quadrature serves the plan.
constexpr double kSurrogateBound = 1e-5;

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

int validate_medium(int32_t L, const std::vector<double>& d, const std::vector<double>& eps) {
  if (L < 1 || L > kMaxL) return FMMLM_EINVAL;
  for (int i = 0; i < L; ++i) {
    if (!std::isfinite(d[i])) return FMMLM_EINTERFACES;
    if (i > 0 && !(d[i] < d[i - 1])) return FMMLM_EINTERFACES;
  }
  for (int i = 0; i <= L; ++i)
    if (!std::isfinite(eps[i]) || !(eps[i] > 0.0)) return FMMLM_EEPS;
  return FMMLM_OK;
}

Medium make_medium(int L, const double* d, const double* eps) {
  Medium md;
  std::memset(&md, 0, sizeof(md));
  md.L = L;
  for (int i = 0; i < L; ++i) md.d[i] = d[i];
  for (int i = 0; i <= L; ++i) md.eps[i] = eps[i];
  for (int i = 0; i <= kMaxL; ++i) md.acoef[i] = 1.0;
  return md;
}

// The general interface conditions (coefficients a, b): eps = b / a, acoef = a.
Medium make_medium_ab(int L, const double* d, const double* a, const double* b) {
  Medium md;
  std::memset(&md, 0, sizeof(md));
  md.L = L;
  for (int i = 0; i < L; ++i) md.d[i] = d[i];
  for (int i = 0; i <= kMaxL; ++i) md.acoef[i] = 1.0;
  for (int i = 0; i <= L; ++i) {
    md.eps[i] = b[i] / a[i];
    md.acoef[i] = a[i];
  }
  return md;
}

double coefA_host(int n, int m) {
  const double cn = std::sqrt((2.0 * n + 1.0) / (4.0 * M_PI));
  return ((n & 1) ? -1.0 : 1.0) * cn / std::sqrt(std::tgamma(n - m + 1.0) * std::tgamma(n + m + 1.0));
}

void drop_graph(fmmlm_plan_s* P) {
  if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
  P->gexec = nullptr;
  P->gkey = GraphKey{};
}

void free_plan(fmmlm_plan_s* P) {
  if (!P) return;
  drop_graph(P);
  for (hipEvent_t e : {P->ev_q, P->ev_m, P->ev_near, P->ev_top, P->ev_l, P->ev_done})
    if (e) (void)hipEventDestroy(e);
  for (hipStream_t q : {P->s_near, P->s_top})
    if (q) (void)hipStreamDestroy(q);
  for (auto e : P->prof_ev) (void)hipEventDestroy(e);
  for (auto& b : P->bufs) hipFree(b.ptr);
  delete P;
}

// The quadrature judges the learned form: up to 256 tasks spread over the
// list are recomputed without it.  A task's error is R1 max_{N,M} 0.87^N
// |S^N I_{N,M} (learned) - S^N I_{N,M} (quadrature)|, R1 = |(rho, z + zinf)|:
// relative to the interaction 1/R1 that the task's operator carries, with the
// weight (0.87)^N that the scaled expansions of two boxes (radius at most
// 0.87 S) put on degree N.  The largest goes to the plan's stats.
int surrogate_check(fmmlm_plan_s* P, const std::vector<CompInfo>& comps, const std::vector<SommTask>& tasks,
                    const double* d_tables, hipStream_t st) {
  const int64_t nt = (int64_t)tasks.size();
  const int64_t k = std::min<int64_t>(nt, 256);
  if (k == 0) return FMMLM_OK;
  std::vector<SommTask> pick(k);
  std::vector<int64_t> idx(k);
  for (int64_t i = 0; i < k; ++i) {
    idx[i] = i * nt / k;
    pick[i] = tasks[idx[i]];
  }
  const size_t per = (size_t)P->ng;
  const int nmax = 2 * P->p;
  double* dq = nullptr;
  FMM_HIP_TRY(hipMalloc(&dq, k * per * sizeof(double)));
  int rc = gpu_sommerfeld_tables(P->medium, comps, pick, nmax, dq, st);
  std::vector<double> q(k * per), g(k * per);
  if (rc == FMMLM_OK) {
    hipError_t e = hipMemcpy(q.data(), dq, k * per * sizeof(double), hipMemcpyDeviceToHost);
    for (int64_t i = 0; i < k && e == hipSuccess; ++i)
      e = hipMemcpy(g.data() + i * per, d_tables + idx[i] * per, per * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      set_last_error(hipGetErrorString(e));
      rc = FMMLM_EDEVICE;
    }
  }
  hipFree(dq);
  if (rc) return rc;
  double worst = 0.0;
  for (int64_t i = 0; i < k; ++i) {
    const SommTask& tk = pick[i];
    const double Z1 = tk.z + comps[tk.comp].zinf;
    const double R1 = std::sqrt(tk.rho * tk.rho + Z1 * Z1);
    double w = R1;
    for (int n = 0; n <= nmax; ++n, w *= 0.87)
      for (int m = 0; m <= n; ++m) {
        const size_t j = (size_t)n * (n + 1) / 2 + m;
        worst = std::max(worst, w * std::fabs(q[i * per + j] - g[i * per + j]));
      }
  }
  P->stats.surrogate_check = worst;
  return FMMLM_OK;
}

// A batched pass costs about the same at any width (its kernels run 64 lanes a
// vector block), so narrow passes are slower than evaluating their vectors one
// by one.  Time one single-vector evaluation and one batched pass of gmax
// vectors (zero charges; best of three after a warm-up) and set the width from
// which a batched pass pays.
static int tune_batch_width(fmmlm_plan_s* P, hipStream_t st) {
  P->batch_min = 2;
  P->stats.batch_min_rhs = 2;
  if (P->gmax < 2) return FMMLM_OK;
  const size_t bytes = (size_t)P->N * (size_t)P->gmax * sizeof(double);
  double *q = nullptr, *phi = nullptr;
  FMM_HIP_TRY(hipMalloc(&q, bytes));
  if (hipMalloc(&phi, bytes) != hipSuccess) {
    (void)hipFree(q);
    return FMMLM_ENOMEM;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = FMMLM_OK;
  if (hipMemsetAsync(q, 0, bytes, st) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess)
    rc = FMMLM_EDEVICE;
  auto best_ms = [&](bool batched) -> double {
    double tmin = 1e300;
    for (int rep = 0; rep < 4 && rc == FMMLM_OK; ++rep) {
      (void)hipEventRecord(e0, st);
      rc = batched ? gpu_eval_batch(P, P->gmax, q, P->N, phi, P->N, FMMLM_FREE | FMMLM_REACTION, st, nullptr)
                   : gpu_eval_one(P, q, phi, FMMLM_FREE | FMMLM_REACTION, st, nullptr);
      (void)hipEventRecord(e1, st);
      if (rc) break;
      if (hipEventSynchronize(e1) != hipSuccess) {
        rc = FMMLM_EDEVICE;
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) tmin = std::min(tmin, (double)ms);
    }
    return tmin;
  };
  const double t1 = best_ms(false);
  const double tb = best_ms(true);
  if (rc == FMMLM_OK && t1 > 0.0 && tb < 1e300) {
    const double w = std::ceil(tb / t1);
    P->batch_min = (int)std::max(2.0, std::min(w, (double)P->gmax + 1.0));
    P->stats.batch_min_rhs = P->batch_min;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(q);
  (void)hipFree(phi);
  return rc;
}

int build_plan(fmmlm_plan_s* P, const std::vector<double>& X, const std::vector<double>& Y,
               const std::vector<double>& Z, const std::vector<int32_t>& LAY, hipStream_t st) {
  const int L = P->L;
  const int64_t N = P->N;
  auto tphase = std::chrono::steady_clock::now();
  // ---- anchored trees (layer, side) with members in user order
  std::vector<std::vector<int64_t>> members(L + 1);
  for (int64_t i = 0; i < N; ++i) members[LAY[i]].push_back(i);
  for (int l = 0; l <= L; ++l) {
    if (members[l].empty()) continue;
    for (int side = 1; side <= 2; ++side) {
      if (side == 1 && l > L - 1) continue;
      if (side == 2 && l < 1) continue;
      TreeInfo t;
      t.layer = l;
      t.side = side;
      t.n = (int64_t)members[l].size();
      P->trees.push_back(t);
    }
  }
  const int nt = (int)P->trees.size();
  // ---- common frame
  double xmin = X[0], xmax = X[0], ymin = Y[0], ymax = Y[0], hmax = 0.0, hmin = INFINITY;
  for (int64_t i = 0; i < N; ++i) {
    xmin = std::min(xmin, X[i]);
    xmax = std::max(xmax, X[i]);
    ymin = std::min(ymin, Y[i]);
    ymax = std::max(ymax, Y[i]);
    const int l = LAY[i];
    if (l <= L - 1) {
      hmax = std::max(hmax, Z[i] - P->d[l]);
      hmin = std::min(hmin, Z[i] - P->d[l]);
    }
    if (l >= 1) {
      hmax = std::max(hmax, P->d[l - 1] - Z[i]);
      hmin = std::min(hmin, P->d[l - 1] - Z[i]);
    }
  }
  P->x0 = xmin;
  P->y0 = ymin;
  P->W = std::max(std::max(xmax - xmin, ymax - ymin), hmax) * (1.0 + std::ldexp(1.0, -20));
  if (!(hmin > 1e-12 * P->W)) return FMMLM_EONINTERFACE;
  P->scale = std::ldexp(1.0, 21) / P->W;
  // ---- keys + sort on the GPU
  double *dx = nullptr, *dy = nullptr, *dz = nullptr;
  FMM_HIP_TRY(hipMalloc(&dx, N * 8));
  FMM_HIP_TRY(hipMalloc(&dy, N * 8));
  FMM_HIP_TRY(hipMalloc(&dz, N * 8));
  FMM_HIP_TRY(hipMemcpyAsync(dx, X.data(), N * 8, hipMemcpyHostToDevice, st));
  FMM_HIP_TRY(hipMemcpyAsync(dy, Y.data(), N * 8, hipMemcpyHostToDevice, st));
  FMM_HIP_TRY(hipMemcpyAsync(dz, Z.data(), N * 8, hipMemcpyHostToDevice, st));
  int64_t off = 0;
  for (int t = 0; t < nt; ++t) {
    TreeInfo& T = P->trees[t];
    T.pt_off = off;
    off += T.n;
    T.keys.resize(T.n);
    T.perm = members[T.layer];
    const double dref = (T.side == 1) ? P->d[T.layer] : P->d[T.layer - 1];
    std::string err;
    int rc = gpu_sort_tree(dx, dy, dz, T.n, T.side, dref, P->x0, P->y0, P->scale, T.keys.data(),
                           T.perm.data(), st, &err);
    if (rc) {
      hipFree(dx);
      hipFree(dy);
      hipFree(dz);
      return rc;
    }
  }
  hipFree(dx);
  hipFree(dy);
  hipFree(dz);
  P->NP = off;
  P->stats.tree_seconds = seconds_since(tphase);
  tphase = std::chrono::steady_clock::now();
  // ---- boxes, level by level over all trees (level-major global order)
  Builder B;
  B.P = P;
  const int cap = P->opts.leaf_cap;
  std::vector<std::vector<int>> per_level;  // global ids per level
  B.root.assign(nt, -1);
  per_level.emplace_back();
  for (int t = 0; t < nt; ++t) {
    HBox r{0, 0, t, P->trees[t].pt_off, P->trees[t].n, -1, -1, 0, 0, 0, 0};
    B.root[t] = (int)B.boxes.size();
    per_level[0].push_back((int)B.boxes.size());
    B.boxes.push_back(r);
  }
  // A box is split when it holds more than cap points, and also when a box
  // that the traversal would pair with it at this level (free: same tree,
  // adjacent or inside the MAC; reaction: any tree, touching-interface
  // adjacency or inside the MAC in the mirrored frame) holds more than
  // kBalance * cap points.  Without the second rule a sparse leaf would take
  // the P2P of a whole dense subtree next to it (unbounded pair counts when
  // densities differ across layers or clusters); with it a leaf's P2P partner
  // holds at most kBalance * cap points.
  constexpr int64_t kBalance = 8;
  const int mac = P->opts.mac_d2;
  std::vector<char> free_tree(nt);
  for (int t = 0; t < nt; ++t) {
    const TreeInfo& T = P->trees[t];
    free_tree[t] = (T.layer <= L - 1) ? (T.side == 1) : (T.side == 2);
  }
  auto cell = [](int ix, int iy, int ih) {
    return spread1by2((uint64_t)ix) | (spread1by2((uint64_t)iy) << 1) | (spread1by2((uint64_t)ih) << 2);
  };
  for (int l = 0;; ++l) {
    std::vector<int> next;
    std::vector<char> split(per_level[l].size(), 0);
    if (l < kMaxLevel) {
      std::unordered_set<uint64_t> heavy_reac;               // cells (any tree), ih <= 2
      std::vector<std::unordered_set<uint64_t>> heavy_free(nt);
      for (size_t k = 0; k < per_level[l].size(); ++k) {
        const HBox& bx = B.boxes[per_level[l][k]];
        if (bx.count <= cap) continue;
        split[k] = 1;
        if (bx.count <= kBalance * cap) continue;
        if (compact1by2(bx.prefix >> 2) <= 2) heavy_reac.insert(bx.prefix);
        if (free_tree[bx.tree]) heavy_free[bx.tree].insert(bx.prefix);
      }
      const int n1d = 1 << l;
      for (size_t k = 0; k < per_level[l].size(); ++k) {
        if (split[k]) continue;
        const HBox& bx = B.boxes[per_level[l][k]];
        const int ix = compact1by2(bx.prefix), iy = compact1by2(bx.prefix >> 1), ih = compact1by2(bx.prefix >> 2);
        bool hit = false;
        for (int dx = -3; dx <= 3 && !hit; ++dx)
          for (int dy = -3; dy <= 3 && !hit; ++dy) {
            const int jx = ix + dx, jy = iy + dy;
            if (jx < 0 || jy < 0 || jx >= n1d || jy >= n1d) continue;
            if (!heavy_reac.empty()) {
              for (int jh = 0; jh <= 2 && !hit; ++jh) {
                const int dz = ih + jh + 1;
                const bool near = (std::abs(dx) <= 1 && std::abs(dy) <= 1 && dz == 1) ||
                                  dx * dx + dy * dy + dz * dz < mac;
                if (near && heavy_reac.count(cell(jx, jy, jh))) hit = true;
              }
            }
            if (free_tree[bx.tree] && !heavy_free[bx.tree].empty()) {
              for (int dz = -3; dz <= 3 && !hit; ++dz) {
                const int jh = ih + dz;
                if (jh < 0 || jh >= n1d) continue;
                const bool near = (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) ||
                                  dx * dx + dy * dy + dz * dz < mac;
                if (near && heavy_free[bx.tree].count(cell(jx, jy, jh))) hit = true;
              }
            }
          }
        split[k] = hit;
      }
    }
    for (size_t k = 0; k < per_level[l].size(); ++k) {
      const int b = per_level[l][k];
      const HBox parent = B.boxes[b];  // copy: the vector grows below
      if (!split[k]) continue;
      const TreeInfo& T = P->trees[parent.tree];
      const int shift = 3 * (20 - l);
      int64_t i = parent.start;
      const int64_t e = parent.start + parent.count;
      const int first_child = (int)B.boxes.size();
      int nch = 0;
      while (i < e) {
        const unsigned dg = (unsigned)((T.keys[i - T.pt_off] >> shift) & 7u);
        int64_t j = i;
        while (j < e && (unsigned)((T.keys[j - T.pt_off] >> shift) & 7u) == dg) ++j;
        HBox c{(parent.prefix << 3) | dg, l + 1, parent.tree, i, j - i, b, -1, 0, 0, 0, 0};
        next.push_back((int)B.boxes.size());
        B.boxes.push_back(c);
        ++nch;
        i = j;
      }
      B.boxes[b].child0 = first_child;
      B.boxes[b].nchild = nch;
    }
    if (next.empty()) break;
    per_level.push_back(next);
  }
  // children were appended in level order, trees in order, so ids are level-major.
  P->maxlev = (int)per_level.size() - 1;
  P->lev_off.assign(P->maxlev + 2, 0);
  for (int l = 0; l <= P->maxlev; ++l) P->lev_off[l + 1] = P->lev_off[l] + (int64_t)per_level[l].size();
  P->NB = (int64_t)B.boxes.size();
  if (P->NB >= (int64_t)1 << 30) return FMMLM_ENOMEM;
  for (auto& bx : B.boxes) {
    uint64_t pf = bx.prefix;
    bx.ix = compact1by2(pf);
    bx.iy = compact1by2(pf >> 1);
    bx.ih = compact1by2(pf >> 2);
  }
  // ---- interaction lists
  B.free_code_to_op.assign(15 * 15 * 15, -1);
  B.mac_d2 = P->opts.mac_d2;
  B.p2p_free.resize(P->NB);
  B.p2p_reac.resize(P->NB);
  for (int t = 0; t < nt; ++t) {
    const TreeInfo& T = P->trees[t];
    const bool free_tree = (T.layer <= L - 1) ? (T.side == 1) : (T.side == 2);
    if (free_tree) B.process_free(B.root[t], B.root[t]);
  }
  std::vector<CompInfo> comps;
  for (int t = 0; t < nt; ++t)
    for (int s = 0; s < nt; ++s) {
      comps.push_back(make_comp(P->medium, P->trees[t].layer, P->trees[s].layer, P->trees[t].side,
                                P->trees[s].side));
    }
  const fmmlm_surrogate_s* sur = P->opts.surrogate;
  std::vector<int32_t> smap;  // plan component -> surrogate component
  if (sur) {
    for (int t = 0; t < nt; ++t)
      for (int s = 0; s < nt; ++s) {
        const TreeInfo& A = P->trees[t];
        const TreeInfo& S = P->trees[s];
        smap.push_back(side_index(L, A.layer, A.side) * 2 * L + side_index(L, S.layer, S.side));
      }
  }
  for (int t = 0; t < nt; ++t)
    for (int s = 0; s < nt; ++s) B.process_reac(B.root[t], B.root[s], t * nt + s);
  // ---- leaves
  std::vector<int32_t> leaves;
  for (int64_t b = 0; b < P->NB; ++b)
    if (B.boxes[b].nchild == 0) leaves.push_back((int32_t)b);
  P->nleaves = (int64_t)leaves.size();
  // ---- box arrays
  std::vector<double> bcx(P->NB), bcy(P->NB), bch(P->NB);
  std::vector<int32_t> blevel(P->NB), bstart(P->NB), bcount(P->NB), bparent(P->NB), bchild0(P->NB), bnchild(P->NB);
  for (int64_t b = 0; b < P->NB; ++b) {
    const HBox& bx = B.boxes[b];
    const double S = P->W / std::ldexp(1.0, bx.level);
    bcx[b] = P->x0 + (bx.ix + 0.5) * S;
    bcy[b] = P->y0 + (bx.iy + 0.5) * S;
    bch[b] = (bx.ih + 0.5) * S;
    blevel[b] = bx.level;
    bstart[b] = (int32_t)bx.start;
    bcount[b] = (int32_t)bx.count;
    bparent[b] = bx.parent;
    bchild0[b] = bx.child0;
    bnchild[b] = bx.nchild;
  }
  // ---- M2L CSR: per target, free entries first, then reaction, in traversal order
  const int64_t ne = (int64_t)B.m_tgt.size();
  if (ne >= (int64_t)1 << 31) return FMMLM_ENOMEM;
  std::vector<int32_t> mptr(P->NB + 1, 0), mnfree(P->NB, 0);
  for (int64_t e = 0; e < ne; ++e) {
    mptr[B.m_tgt[e] + 1]++;
    if (B.m_isfree[e]) mnfree[B.m_tgt[e]]++;
  }
  for (int64_t b = 0; b < P->NB; ++b) mptr[b + 1] += mptr[b];
  std::vector<int32_t> msrc(ne), mop(ne);
  {
    std::vector<int32_t> fill_free(P->NB), fill_reac(P->NB);
    for (int64_t b = 0; b < P->NB; ++b) {
      fill_free[b] = mptr[b];
      fill_reac[b] = mptr[b] + mnfree[b];
    }
    const int nfreeops = (int)(B.free_off.size() / 3);
    int64_t nfree_pairs = 0, nreac_pairs = 0;
    for (int64_t e = 0; e < ne; ++e) {
      const int tg = B.m_tgt[e];
      int32_t pos;
      int32_t op;
      if (B.m_isfree[e]) {
        pos = fill_free[tg]++;
        op = B.m_op[e];
        ++nfree_pairs;
      } else {
        pos = fill_reac[tg]++;
        op = ~(nfreeops + B.m_op[e]);  // mirrored source
        ++nreac_pairs;
      }
      msrc[pos] = B.m_src[e];
      mop[pos] = op;
    }
    P->stats.m2l_free_pairs = nfree_pairs;
    P->stats.m2l_reaction_pairs = nreac_pairs;
    P->n_free_ops = nfreeops;
    P->nops = nfreeops + (int64_t)B.reac_task.size();
  }
  // ---- M2L steps: the top levels (few boxes, many distinct operators) go to
  // the sparse FP64 kernel, the levels below them operator-major: chunks of up
  // to tile_cols targets of a group of operators, each a tile of its own
  std::vector<int32_t> tptr(1, 0), ttgt, tlev, sop, skind, ssrc, smask, us, umask, tuptr;
  {
    {
      const int nr0 = (P->p + 1) * (P->p + 1);
      const int mr0 = (nr0 + 31) / 32;
      P->mrt = (mr0 + 1) / 2 * 2;
      if (P->mrt < 2) P->mrt = 2;
      P->nrk = (nr0 + 15) / 16 * 16;
      P->tile_cols = (P->mrt <= 4) ? 128 : 64;
    }
    const int TBc = P->tile_cols;
    const int nfo = (int)P->n_free_ops;
    const int ksp = P->opts.fp64_top_levels;  // levels of the sparse kernel
    {
      std::vector<int32_t> spb;
      for (int l = 0; l < std::min(ksp, P->maxlev + 1); ++l)
        for (int64_t b = P->lev_off[l]; b < P->lev_off[l + 1]; ++b)
          if (mptr[b + 1] > mptr[b]) {
            spb.push_back((int32_t)b);
            P->stats.m2l_top_pairs += mptr[b + 1] - mptr[b];
          }
      P->n_sp_boxes = (int64_t)spb.size();
      if (int rc0 = dev_upload(P, &P->sp_boxes, spb, st)) return rc0;
      // work items: runs of kSpItemRounds rounds of sp_ne entries (the block's
      // threads hold sp_ne entries x the coefficients (n, m >= 0) in groups of
      // four orders; LDS holds their source expansions and operator tables,
      // then their sums, at most 60 KiB)
      const int nc = P->nc, ng = P->ng, nr = (P->p + 1) * (P->p + 1);
      int tps = 0;
      for (int n = 0; n <= P->p; ++n) tps += (n + 4) / 4;
      P->sp_ne = std::max(1, std::min(kSpThreads / tps, 61440 / (std::max(nr + ng, nc) * 16)));
      P->sp_threads = (P->sp_ne * tps + 63) / 64 * 64;
      const int run = kSpItemRounds * P->sp_ne;
      std::vector<int32_t> items, iptr(1, 0);
      for (const int32_t b : spb) {
        for (int32_t e = mptr[b]; e < mptr[b + 1]; e += run) {
          items.push_back(b);
          items.push_back(e);
          items.push_back(std::min<int32_t>(e + run, mptr[b + 1]));
        }
        iptr.push_back((int32_t)(items.size() / 3));
      }
      P->n_sp_items = (int64_t)(items.size() / 3);
      if (int rc0 = dev_upload(P, &P->sp_items, items, st)) return rc0;
      if (int rc0 = dev_upload(P, &P->sp_item_ptr, iptr, st)) return rc0;
      if (int rc0 = dev_alloc(P, &P->Psp, (size_t)std::max<int64_t>(P->n_sp_items, 1) * nc * 2)) return rc0;
    }
    for (int grp = 0; grp <= 4; ++grp) P->tile_grp[grp] = 0;  // no target tiles (M2L is operator-major)
    // Levels below the sparse ones: operator-major chunks (FP32 products on the
    // FP32 form's matrix-core kernel, FP64 ones on the FP64 tile GEMM).  The
    // operators are taken kM2LGroupOps at a time in operator order (in box units
    // a free-space operator serves every level); the targets that every
    // operator of the group reaches are taken TBc at a time as one chunk whose
    // steps are the group's operators, each with its own sources, so the chunk
    // stores one partial sum per target for all of them.  The rest of each
    // operator's pairs form one-step chunks.  A target appears at most once per
    // operator, so a chunk's columns are distinct targets.  Each target's outputs
    // are then summed over its slots (chunk, column) in chunk order by
    // m2l_slot_reduce_kernel.
    {
      std::vector<std::array<int32_t, 3>> pr;  // (operator, target, source)
      for (int l = ksp; l <= P->maxlev; ++l)
        for (int64_t b = P->lev_off[l]; b < P->lev_off[l + 1]; ++b)
          for (int32_t e = mptr[b]; e < mptr[b + 1]; ++e)
            pr.push_back({(mop[e] >= 0) ? mop[e] : ~mop[e], (int32_t)b, msrc[e]});
      std::sort(pr.begin(), pr.end());
      std::vector<std::pair<size_t, size_t>> oprng;  // each operator's pairs [i0, i1) in pr
      std::vector<uint64_t> opclass;                 // ... and its class (after the sort below)
      for (size_t i0 = 0; i0 < pr.size();) {
        size_t i1 = i0;
        while (i1 < pr.size() && pr[i1][0] == pr[i0][0]) ++i1;
        oprng.push_back({i0, i1});
        i0 = i1;
      }
      // operators in classes that reach the same targets, so that a group's
      // operators share most of them.  Free space: a box meets offset component
      // +3 (or -3) along an axis only from one child position of its parent, so
      // the operators of one such class reach the same targets (the boundary
      // aside).  Reaction operators (after the free ones) by level, offset and
      // component: the components of one offset often hold the same pairs.
      {
        std::vector<uint64_t> rkey((size_t)(P->nops - nfo), 0);
        for (const auto& kv : B.reac_op_id) {
          const int comp = std::get<0>(kv.first), lvl = std::get<1>(kv.first);
          const int dx = std::get<2>(kv.first), dy = std::get<3>(kv.first), dz = std::get<4>(kv.first);
          rkey[kv.second] = ((uint64_t)lvl << 40) | ((uint64_t)(dz & 0xff) << 32) | ((uint64_t)(dx & 0xff) << 24) |
                            ((uint64_t)(dy & 0xff) << 16) | (uint64_t)(comp & 0xffff);
        }
        auto key = [&](int op) -> uint64_t {
          if (op >= nfo) return (uint64_t(1) << 63) | rkey[op - nfo];
          uint64_t c = 0;
          for (int a = 0; a < 3; ++a) {
            const int v = B.free_off[3 * op + a];
            c = 3 * c + (v >= 3 ? 1 : (v <= -3 ? 2 : 0));
          }
          return c;
        };
        std::stable_sort(oprng.begin(), oprng.end(), [&](const std::pair<size_t, size_t>& x,
                                                         const std::pair<size_t, size_t>& y) {
          return key(pr[x.first][0]) < key(pr[y.first][0]);
        });
        // a group holds operators of one class (reaction: one offset)
        for (const auto& r : oprng) {
          const uint64_t k = key(pr[r.first][0]);
          opclass.push_back((k >> 63) ? (k & ~(uint64_t)0xffff) : k);
        }
      }
      std::vector<std::vector<int32_t>> tslots(P->NB);
      std::vector<char> done(pr.size(), 0);
      std::vector<int32_t> hits(P->NB, 0);
      // one chunk: columns c < nc_ hold targets tg[c]; step k applies operator
      // ops[k] to sources src[k][c]
      auto add_chunk = [&](const std::vector<int32_t>& ops, const std::vector<int32_t>& tg,
                           const std::vector<std::vector<int32_t>>& src) {
        const int32_t unit = (int32_t)tlev.size();  // one unit per chunk
        tlev.push_back(B.boxes[tg[0]].level);
        uint32_t msk = 0;
        for (size_t c = 0; c < (size_t)TBc; ++c) {
          const bool on = c < tg.size();
          ttgt.push_back(on ? tg[c] : -1);
          if (on) {
            msk |= 1u << (c >> 3);
            tslots[tg[c]].push_back(unit * TBc + (int32_t)c);
          }
        }
        for (size_t k = 0; k < ops.size(); ++k) {
          for (size_t c = 0; c < (size_t)TBc; ++c) ssrc.push_back(c < tg.size() ? src[k][c] : -1);
          sop.push_back(ops[k]);
          skind.push_back(ops[k] < nfo ? (int32_t)FMMLM_FREE : (int32_t)FMMLM_REACTION);
          smask.push_back((int32_t)msk);
        }
        tptr.push_back((int32_t)sop.size());
      };
      for (size_t g0 = 0, g1 = 0; g0 < oprng.size(); g0 = g1) {
        g1 = g0 + 1;
        while (g1 < oprng.size() && g1 - g0 < (size_t)kM2LGroupOps && opclass[g1] == opclass[g0]) ++g1;
        // (a group whose operator reaches one target twice is not grouped)
        bool distinct = true;
        for (size_t o = g0; o < g1 && distinct; ++o)
          for (size_t i = oprng[o].first + 1; i < oprng[o].second; ++i)
            if (pr[i][1] == pr[i - 1][1]) distinct = false;
        if (g1 - g0 > 1 && distinct) {
          for (size_t o = g0; o < g1; ++o)
            for (size_t i = oprng[o].first; i < oprng[o].second; ++i) ++hits[pr[i][1]];
          // pairs of the group's targets common to all its operators, per
          // operator in target order (each list is sorted by target)
          std::vector<std::vector<size_t>> com(g1 - g0);
          for (size_t o = g0; o < g1; ++o)
            for (size_t i = oprng[o].first; i < oprng[o].second; ++i)
              if (hits[pr[i][1]] == (int32_t)(g1 - g0)) com[o - g0].push_back(i);
          for (size_t o = g0; o < g1; ++o)
            for (size_t i = oprng[o].first; i < oprng[o].second; ++i) hits[pr[i][1]] = 0;
          const size_t ncom = com[0].size();
          if (ncom >= (size_t)kM2LGroupMinTargets) {
            std::vector<int32_t> ops;
            for (size_t o = g0; o < g1; ++o) ops.push_back(pr[oprng[o].first][0]);
            for (size_t c0 = 0; c0 < ncom; c0 += TBc) {
              const size_t n_ = std::min<size_t>(TBc, ncom - c0);
              std::vector<int32_t> tg(n_);
              std::vector<std::vector<int32_t>> src(g1 - g0, std::vector<int32_t>(n_));
              for (size_t c = 0; c < n_; ++c) {
                tg[c] = pr[com[0][c0 + c]][1];
                for (size_t k = 0; k < g1 - g0; ++k) {
                  const size_t i = com[k][c0 + c];
                  if (pr[i][1] != tg[c]) {
                    set_last_error("internal: M2L operator group targets out of step");
                    return FMMLM_EUNSUPPORTED;
                  }
                  src[k][c] = pr[i][2];
                  done[i] = 1;
                }
              }
              add_chunk(ops, tg, src);
            }
          }
        }
        // the group's other pairs, operator by operator
        for (size_t o = g0; o < g1; ++o) {
          std::vector<size_t> rest;
          for (size_t i = oprng[o].first; i < oprng[o].second; ++i)
            if (!done[i]) rest.push_back(i);
          for (size_t c0 = 0; c0 < rest.size(); c0 += TBc) {
            const size_t n_ = std::min<size_t>(TBc, rest.size() - c0);
            std::vector<int32_t> tg(n_);
            std::vector<std::vector<int32_t>> src(1, std::vector<int32_t>(n_));
            for (size_t c = 0; c < n_; ++c) {
              tg[c] = pr[rest[c0 + c]][1];
              src[0][c] = pr[rest[c0 + c]][2];
            }
            add_chunk({pr[oprng[o].first][0]}, tg, src);
          }
        }
      }
      P->tile_grp[3] = P->tile_grp[4] = (int64_t)tlev.size();
      std::vector<int32_t> sbox, sptr(1, 0), slots;
      for (int64_t b = 0; b < P->NB; ++b)
        if (!tslots[b].empty()) {
          sbox.push_back((int32_t)b);
          slots.insert(slots.end(), tslots[b].begin(), tslots[b].end());
          sptr.push_back((int32_t)slots.size());
        }
      P->n_slot_boxes = (int64_t)sbox.size();
      int rc0;
      if ((rc0 = dev_upload(P, &P->slot_boxes, sbox, st)) || (rc0 = dev_upload(P, &P->slot_ptr, sptr, st)) ||
          (rc0 = dev_upload(P, &P->slots, slots, st)))
        return rc0;
    }
    P->ntiles = (int64_t)tlev.size();
    P->nsteps = (int64_t)sop.size();
    P->stats.m2l_steps = P->nsteps;
    P->stats.m2l_chunks = P->ntiles;
    P->stats.m2l_tile_cols = TBc;
    // work units: one per chunk (a chunk has at most kM2LGroupOps steps);
    // unit_split is 0 (no target tiles)
    constexpr int kStepsPerUnit = 16;
    tuptr.assign(1, 0);
    for (int64_t t = 0; t < P->ntiles; ++t) {
      if (t == P->tile_grp[2]) P->unit_split = (int64_t)(us.size() / 2);
      for (int32_t a = tptr[t]; a < tptr[t + 1]; a += kStepsPerUnit) {
        const int32_t b = std::min(a + kStepsPerUnit, tptr[t + 1]);
        us.push_back(a);
        us.push_back(b);
        int32_t um = 0;  // column groups any step of the unit touches
        for (int32_t q = a; q < b; ++q) um |= smask[q];
        umask.push_back(um);
      }
      tuptr.push_back((int32_t)(us.size() / 2));
    }
    if (P->ntiles == P->tile_grp[2]) P->unit_split = (int64_t)(us.size() / 2);
    P->nunits = (int64_t)(us.size() / 2);
    // the chunk units in 8 contiguous ranges of about equal steps, one per XCD
    // (contiguous, so that the chunks of one operator share an XCD's L2)
    {
      const int64_t u0 = P->unit_split, n = P->nunits - u0;
      const int64_t tot = n > 0 ? (int64_t)us[2 * (P->nunits - 1) + 1] - us[2 * u0] : 0;
      int64_t u = 0, acc = 0;
      P->m2l_xcd.off[0] = 0;
      P->m2l_xcd_len = 0;
      for (int x = 1; x <= 8; ++x) {
        const int64_t goal = tot * x / 8;
        while (u < n && acc + (us[2 * (u0 + u) + 1] - us[2 * (u0 + u)]) <= goal) {
          acc += us[2 * (u0 + u) + 1] - us[2 * (u0 + u)];
          ++u;
        }
        if (x == 8) u = n;
        P->m2l_xcd.off[x] = (int32_t)u;
        P->m2l_xcd_len = std::max<int32_t>(P->m2l_xcd_len, P->m2l_xcd.off[x] - P->m2l_xcd.off[x - 1]);
      }
    }
    // each chunk is one unit (the slots index units by chunk)
    if (P->nunits != P->ntiles || P->unit_split != 0) {
      set_last_error("internal: M2L chunks and units differ");
      return FMMLM_EUNSUPPORTED;
    }
    // operator tables must fit a budget (FP64 + FP32 copies)
    const double tbytes = (double)P->nops * P->nrk * 32.0 * P->mrt * (P->fp32 ? 12.0 : 8.0);
    if (tbytes > 32.0 * (1 << 30)) {
      set_last_error("M2L operator tables exceed 32 GiB");
      return FMMLM_ENOMEM;
    }
  }
  // ---- M2M / L2L as GEMMs over tiles of up to xl_tile_cols target boxes of one
  // level: M2M tiles hold parents (one step per child octant present, source
  // = that child, operator = octant; at most 8 units a tile, summed by the
  // kernel's block in unit order); L2L tiles hold children of one octant (one
  // step, source = the parent, operator 8 + octant), so an L2L tile is one
  // unit, whose product is added into the children directly.
  {
    // narrow tiles: a level's translations are few, so more and smaller blocks
    const int TBc = P->xl_tile_cols;
    std::vector<int32_t> xop, xsrc, xus, xumask, xtuptr(1, 0), xtgt, xlev;
    auto add_tile = [&](int l, const std::vector<int32_t>& tg, const std::vector<std::vector<int32_t>>& src,
                        const std::vector<int>& ops) {
      xlev.push_back(l);
      for (int c = 0; c < TBc; ++c) xtgt.push_back(c < (int)tg.size() ? tg[c] : -1);
      for (size_t k = 0; k < ops.size(); ++k) {
        const int32_t a = (int32_t)xop.size();
        xop.push_back(ops[k]);
        uint32_t msk = 0;
        for (int c = 0; c < TBc; ++c) {
          const int32_t v = c < (int)src[k].size() ? src[k][c] : -1;
          xsrc.push_back(v);
          if (v >= 0) msk |= 1u << (c >> 3);
        }
        xus.push_back(a);
        xus.push_back(a + 1);
        xumask.push_back((int32_t)msk);
      }
      xtuptr.push_back((int32_t)(xus.size() / 2));
    };
    auto octant = [&](int64_t b) {
      const HBox& bx = B.boxes[b];
      return (bx.ix & 1) | ((bx.iy & 1) << 1) | ((bx.ih & 1) << 2);
    };
    P->xl_m2m.assign(P->maxlev + 1, {0, 0, 0, 0});
    P->xl_l2l.assign(P->maxlev + 1, {0, 0, 0, 0});
    for (int l = 0; l <= P->maxlev; ++l) {
      // M2M into the parents of level l
      std::array<int64_t, 4> r{(int64_t)xlev.size(), (int64_t)(xus.size() / 2), 0, 0};
      std::vector<int32_t> par;
      for (int64_t b = P->lev_off[l]; b < P->lev_off[l + 1]; ++b)
        if (B.boxes[b].nchild > 0) par.push_back((int32_t)b);
      for (size_t c0 = 0; c0 < par.size(); c0 += TBc) {
        std::vector<int32_t> tg(par.begin() + c0, par.begin() + std::min(par.size(), c0 + TBc));
        std::vector<std::vector<int32_t>> src(8, std::vector<int32_t>(tg.size(), -1));
        for (size_t c = 0; c < tg.size(); ++c) {
          const HBox& bx = B.boxes[tg[c]];
          for (int k = 0; k < bx.nchild; ++k) src[octant(bx.child0 + k)][c] = bx.child0 + k;
        }
        std::vector<int> ops;  // at most 8 (the translation kernel sums a tile's units in one block)
        std::vector<std::vector<int32_t>> used;
        for (int o = 0; o < 8; ++o)
          if (std::any_of(src[o].begin(), src[o].end(), [](int32_t v) { return v >= 0; })) {
            ops.push_back(o);
            used.push_back(src[o]);
          }
        add_tile(l, tg, used, ops);
      }
      r[2] = (int64_t)xlev.size();
      r[3] = (int64_t)(xus.size() / 2);
      P->xl_m2m[l] = r;
      // L2L into the children of level l
      std::array<int64_t, 4> q{(int64_t)xlev.size(), (int64_t)(xus.size() / 2), 0, 0};
      if (l >= 1) {
        for (int o = 0; o < 8; ++o) {
          std::vector<int32_t> ch;
          for (int64_t b = P->lev_off[l]; b < P->lev_off[l + 1]; ++b)
            if (octant(b) == o) ch.push_back((int32_t)b);
          for (size_t c0 = 0; c0 < ch.size(); c0 += TBc) {
            std::vector<int32_t> tg(ch.begin() + c0, ch.begin() + std::min(ch.size(), c0 + TBc));
            std::vector<std::vector<int32_t>> src(1, std::vector<int32_t>(tg.size()));
            for (size_t c = 0; c < tg.size(); ++c) src[0][c] = B.boxes[tg[c]].parent;
            add_tile(l, tg, src, {8 + o});
          }
        }
      }
      q[2] = (int64_t)xlev.size();
      q[3] = (int64_t)(xus.size() / 2);
      P->xl_l2l[l] = q;
    }
    P->xl_units = (int64_t)(xus.size() / 2);
    // translations whose results nothing reads are skipped: M2M into level l
    // only if some M2L takes a source on level l or above it (through later
    // M2M), L2L out of level l only if level l or a level above it receives an
    // M2L (otherwise its local expansions are zero).  With mac_d2 = 4 the root
    // is in no M2L pair, so M2M into it and L2L out of it go.
    {
      std::vector<char> src_on(P->maxlev + 1, 0), tgt_on(P->maxlev + 1, 0);
      for (int64_t b = 0; b < P->NB; ++b)
        for (int32_t e = mptr[b]; e < mptr[b + 1]; ++e) {
          tgt_on[B.boxes[b].level] = 1;
          src_on[B.boxes[msrc[e]].level] = 1;
        }
      P->xl_need_m2m.assign(P->maxlev + 1, 0);
      P->xl_need_l2l.assign(P->maxlev + 1, 0);
      char needm = 0, hasl = 0;
      for (int l = 0; l <= P->maxlev; ++l) {
        needm = needm || src_on[l];
        P->xl_need_m2m[l] = needm;  // M2M into level l
        if (l >= 1) P->xl_need_l2l[l] = hasl;  // L2L from level l - 1 into level l
        hasl = hasl || tgt_on[l];
      }
    }
    int rc0;
#define UPX(field, vec) if ((rc0 = dev_upload(P, &P->field, vec, st))) return rc0
    UPX(xl_step_op, xop); UPX(xl_step_src, xsrc);
    UPX(xl_unit_s, xus); UPX(xl_unit_mask, xumask); UPX(xl_tile_unit_ptr, xtuptr); UPX(xl_tile_tgt, xtgt);
#undef UPX
  }
  // ---- P2P CSR over leaves
  std::vector<int32_t> pptr(P->nleaves + 1, 0), psrc;
  std::vector<int32_t> rptr(P->nleaves + 1, 0), rsrc;
  std::vector<int64_t> rvoff;
  std::vector<int32_t> rp_t, rp_s, rp_c;
  // reaction rows: entry e's target rows have partial sums at rrow[e] + i;
  // work units of kRPUnitRows rows (entry, first row, target count)
  std::vector<int32_t> rrow, runits, runits16;
  int64_t voff = 0, nrows = 0;
  for (int64_t li = 0; li < P->nleaves; ++li) {
    const int b = leaves[li];
    for (auto& pr : B.p2p_free[b]) {
      psrc.push_back(pr.first);
      psrc.push_back(pr.second);
    }
    pptr[li + 1] = (int32_t)(psrc.size() / 2);
    for (auto& r : B.p2p_reac[b]) {
      const int32_t tcnt = (int32_t)B.boxes[b].count;
      for (int32_t r0 = 0; r0 < tcnt; r0 += kRPUnitRows) {
        runits.push_back((int32_t)rvoff.size());
        runits.push_back(r0);
        runits.push_back(tcnt);
      }
      for (int32_t r0 = 0; r0 < tcnt; r0 += 16) {  // batched FP32 form: 16-row matrix-core tiles
        runits16.push_back((int32_t)rvoff.size());
        runits16.push_back(r0);
        runits16.push_back(tcnt);
      }
      rrow.push_back((int32_t)nrows);
      nrows += tcnt;
      rsrc.push_back(r.start);
      rsrc.push_back(r.count);
      rvoff.push_back(voff);
      for (int64_t i = 0; i < B.boxes[b].count; ++i)
        for (int j = 0; j < r.count; ++j) {
          rp_t.push_back((int32_t)(B.boxes[b].start + i));
          rp_s.push_back(r.start + j);
          rp_c.push_back(r.comp);
        }
      voff += B.boxes[b].count * (int64_t)r.count;
    }
    rptr[li + 1] = (int32_t)(rsrc.size() / 2);
  }
  std::vector<int32_t> plv;
  for (int64_t li = 0; li < P->nleaves; ++li)
    if (pptr[li + 1] > pptr[li]) plv.push_back((int32_t)li);
  P->n_pl_leaves = (int64_t)plv.size();
  // ---- mutual free P2P units.  Every free-space pair of points is in both
  // leaves' lists (the list relation is symmetric); the pair of a leaf A and a
  // list range C is evaluated once, by A's units when C lies after A in tree
  // order (its 1/r serves both sums), and skipped in the units of C's leaves.
  // The leaf's own range stays one way (first range of each unit).  A unit
  // covering leaf c in its later ranges fills one row of c's source-side sums.
  std::vector<int32_t> mleaf, mtb, mrptr(1, 0), mrng, cbn(P->nleaves, -1);
  std::vector<int64_t> mboff, mwork;
  // (unit's first position of the leaf, leaf, row of the leaf)
  std::vector<std::array<int64_t, 3>> segs;
  int64_t npos = 0;
  {
    const int tpb = P->fp32 ? kPLUnitTargetsF32 : kPLUnitTargetsF64;
    std::vector<std::pair<int64_t, int32_t>> lstart;  // (first point, leaf list index)
    for (int64_t li = 0; li < P->nleaves; ++li)
      if (B.boxes[leaves[li]].count > 0) lstart.push_back({B.boxes[leaves[li]].start, (int32_t)li});
    std::sort(lstart.begin(), lstart.end());
    std::vector<std::pair<int64_t, int64_t>> up;
    for (int64_t li = 0; li < P->nleaves; ++li) {
      const HBox& A = B.boxes[leaves[li]];
      if (A.count <= 0 || pptr[li + 1] == pptr[li]) continue;
      up.clear();
      bool self = false;
      for (auto& pr : B.p2p_free[leaves[li]]) {
        if (pr.first == A.start) {
          if (pr.second != A.count) {
            set_last_error("internal: free P2P range at a leaf's start is not the leaf");
            return FMMLM_EUNSUPPORTED;
          }
          self = true;
        } else if (pr.first > A.start) {
          up.push_back({pr.first, pr.second});
        }
      }
      if (!self) {
        set_last_error("internal: leaf without its own free P2P range");
        return FMMLM_EUNSUPPORTED;
      }
      if (cbn[li] < 0) cbn[li] = 0;
      std::sort(up.begin(), up.end());
      std::vector<std::pair<int64_t, int64_t>> merged;  // contiguous ranges joined
      for (auto& r : up) {
        if (!merged.empty() && merged.back().first + merged.back().second == r.first)
          merged.back().second += r.second;
        else
          merged.push_back(r);
      }
      int64_t mtot = 0;
      for (auto& r : merged) mtot += r.second;
      for (int64_t tb = 0; tb < A.count; tb += tpb) {
        const int64_t tcp = std::min<int64_t>(tpb, A.count - tb);
        mleaf.push_back((int32_t)li);
        mtb.push_back((int32_t)tb);
        mrng.push_back((int32_t)A.start);
        mrng.push_back((int32_t)A.count);
        for (auto& r : merged) {
          mrng.push_back((int32_t)r.first);
          mrng.push_back((int32_t)r.second);
        }
        mrptr.push_back((int32_t)(mrng.size() / 2));
        mwork.push_back(tcp * (A.count + mtot));
        mboff.push_back(npos);
        for (auto& r : merged) {
          auto it = std::lower_bound(lstart.begin(), lstart.end(), std::make_pair(r.first, (int32_t)-1));
          int64_t covered = 0;
          for (; it != lstart.end() && it->first < r.first + r.second; ++it) {
            const int32_t c = it->second;
            const int64_t cn = B.boxes[leaves[c]].count;
            if (cbn[c] < 0) cbn[c] = 0;
            segs.push_back({npos + covered, c, cbn[c]++});
            covered += cn;
          }
          if (covered != r.second) {
            set_last_error("internal: free P2P range is not a union of leaves");
            return FMMLM_EUNSUPPORTED;
          }
          npos += r.second;
        }
      }
    }
  }
  P->n_mu_units = (int64_t)mleaf.size();
  P->pl_split = P->n_mu_units;  // all at the fork until the evaluation-level tuner decides
  // launch order: most pairs first, so that the launch does not end on a few
  // long units (each unit writes its own slots: the order leaves results alone)
  std::vector<int32_t> morder(mleaf.size());
  for (size_t u = 0; u < morder.size(); ++u) morder[u] = (int32_t)u;
  std::stable_sort(morder.begin(), morder.end(), [&](int32_t a, int32_t b) { return mwork[a] > mwork[b]; });
  std::vector<int64_t> cbbase(P->nleaves, 0);
  int64_t nbvals = 0;
  for (int64_t li = 0; li < P->nleaves; ++li) {
    cbbase[li] = nbvals;
    if (cbn[li] > 0) nbvals += (int64_t)cbn[li] * B.boxes[leaves[li]].count;
  }
  if (nbvals >= ((int64_t)1 << 31)) {
    set_last_error("free P2P: more than 2^31 source-side sums");
    return FMMLM_EUNSUPPORTED;
  }
  std::vector<int32_t> mbidx(std::max<int64_t>(npos, 1), 0);
  for (auto& sg : segs) {
    const int64_t c = sg[1], cn = B.boxes[leaves[c]].count, base = cbbase[c] + sg[2] * cn;
    for (int64_t i = 0; i < cn; ++i) mbidx[sg[0] + i] = (int32_t)(base + i);
  }
  P->stats.p2p_free_pairs = B.free_pairs;
  P->stats.p2p_reaction_pairs = B.reac_pairs;
  // ---- leaf of every tree point, free-space point ranges
  std::vector<int32_t> pleaf(P->NP, -1);
  for (int64_t li = 0; li < P->nleaves; ++li) {
    const HBox& bx = B.boxes[leaves[li]];
    P->max_leaf = std::max<int64_t>(P->max_leaf, bx.count);
    for (int64_t g = bx.start; g < bx.start + bx.count; ++g) pleaf[g] = (int32_t)li;
  }
  for (int t = 0; t < nt; ++t) {
    const TreeInfo& T = P->trees[t];
    const bool free_tree = (T.layer <= L - 1) ? (T.side == 1) : (T.side == 2);
    if (free_tree) P->free_ranges.push_back({T.pt_off, T.n});
  }
  // ---- points in tree order
  std::vector<double> px(P->NP), py(P->NP), ph(P->NP);
  std::vector<int32_t> puser(P->NP), upos(2 * N, -1);
  for (int t = 0; t < nt; ++t) {
    const TreeInfo& T = P->trees[t];
    const double dref = (T.side == 1) ? P->d[T.layer] : P->d[T.layer - 1];
    for (int64_t k = 0; k < T.n; ++k) {
      const int64_t u = T.perm[k];
      const int64_t g = T.pt_off + k;
      px[g] = X[u];
      py[g] = Y[u];
      ph[g] = (T.side == 1) ? (Z[u] - dref) : (dref - Z[u]);
      puser[g] = (int32_t)u;
      if (upos[2 * u] < 0) upos[2 * u] = (int32_t)g; else upos[2 * u + 1] = (int32_t)g;
    }
  }
  // ---- constants
  const int p = P->p;
  std::vector<double> coefA(ncoef(2 * p));
  for (int n = 0; n <= 2 * p; ++n)
    for (int m = 0; m <= n; ++m) coefA[cidx(n, m)] = coefA_host(n, m);
  std::vector<double> scl(P->maxlev + 1);
  for (int l = 0; l <= P->maxlev; ++l) scl[l] = std::ldexp(1.0, l) / P->W;
  // ---- uploads
  int rc;
#define UP(field, vec) if ((rc = dev_upload(P, &P->field, vec, st))) return rc
  UP(px, px); UP(py, py); UP(ph, ph); UP(puser, puser); UP(user_pos, upos); UP(pleaf, pleaf);
  UP(bcx, bcx); UP(bcy, bcy); UP(bch, bch); UP(blevel, blevel); UP(bstart, bstart); UP(bcount, bcount);
  UP(bparent, bparent); UP(bchild0, bchild0); UP(bnchild, bnchild); UP(leaves, leaves);
  UP(m2l_ptr, mptr); UP(m2l_nfree, mnfree); UP(m2l_src, msrc); UP(m2l_op, mop);
  UP(p2p_ptr, pptr); UP(p2p_src, psrc); UP(pl_leaves, plv); UP(rp_ptr, rptr); UP(rp_src, rsrc); UP(rp_voff, rvoff);
  UP(mu_order, morder); UP(mu_leaf, mleaf); UP(mu_tb, mtb); UP(mu_rptr, mrptr); UP(mu_rng, mrng); UP(mu_boff, mboff);
  UP(mu_bidx, mbidx); UP(cb_base, cbbase); UP(cb_n, cbn);
  if ((rc = dev_alloc(P, &P->mu_a, (size_t)P->NP))) return rc;
  if (P->fp32) {
    float* b32 = nullptr;
    if ((rc = dev_alloc(P, &b32, (size_t)std::max<int64_t>(nbvals, 1)))) return rc;
    P->mu_b = b32;
  } else {
    double* b64 = nullptr;
    if ((rc = dev_alloc(P, &b64, (size_t)std::max<int64_t>(nbvals, 1)))) return rc;
    P->mu_b = b64;
  }
  UP(rp_row, rrow); UP(rp_units, runits);
  P->n_rp_units = (int64_t)(runits.size() / 3);
  if ((rc = dev_alloc(P, &P->Prp, (size_t)std::max<int64_t>(nrows, 1)))) return rc;
  if (P->fp32 && P->opts.max_rhs > 1) {
    UP(rp_units16, runits16);
    P->n_rp_units16 = (int64_t)(runits16.size() / 3);
    if ((rc = dev_alloc(P, &P->Prb, (size_t)std::max<int64_t>(nrows, 1) * 64))) return rc;
  }
  // recurrence coefficients of the regular solid harmonics (P2M, L2P):
  // [cidx(n,m)] a = sqrt((4n^2-1)/(n^2-m^2)), [nc + cidx] b = sqrt(((n-1)^2-m^2)/(4(n-1)^2-1)),
  // [2 nc + m] sqrt((2m+1)/(2m)) (m >= 1), [2 nc + p + 1 + m] sqrt(2m+3)
  std::vector<double> coefR(2 * ncoef(p) + 2 * (p + 1), 0.0);
  {
    const int ncp = ncoef(p);
    for (int n = 0; n <= p; ++n)
      for (int m = 0; m <= n; ++m) {
        if (n >= m + 2) {
          coefR[cidx(n, m)] = std::sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
          coefR[ncp + cidx(n, m)] =
              std::sqrt(((double)(n - 1) * (n - 1) - (double)m * m) / (4.0 * (n - 1) * (n - 1) - 1.0));
        }
      }
    for (int m = 0; m <= p; ++m) {
      coefR[2 * ncp + m] = m > 0 ? std::sqrt((2.0 * m + 1.0) / (2.0 * m)) : 1.0;
      coefR[2 * ncp + p + 1 + m] = std::sqrt(2.0 * m + 3.0);
    }
  }
  UP(coefA, coefA); UP(coefR, coefR); UP(sc_levels, scl);
  UP(tile_ptr, tptr); UP(tile_tgt, ttgt); UP(tile_level, tlev); UP(step_op, sop); UP(step_src, ssrc);
  UP(unit_s, us); UP(tile_unit_ptr, tuptr); UP(step_kind, skind); UP(step_mask, smask); UP(unit_mask, umask);
  if (P->fp32) {
    if ((rc = dev_alloc(P, &P->W32m, (size_t)std::max<int64_t>(P->nunits, 1) * P->tile_cols * 32 * P->mrt)))
      return rc;
  } else if ((rc = dev_alloc(P, &P->Wm2l, (size_t)std::max<int64_t>(P->nunits, 1) * P->tile_cols * 32 * P->mrt))) {
    return rc;
  }
#undef UP
  P->stats.lists_seconds = seconds_since(tphase);
  tphase = std::chrono::steady_clock::now();
  // ---- operators: free-space harmonics and reaction Sommerfeld tables
  if ((rc = dev_alloc(P, &P->G, (size_t)std::max<int64_t>(P->nops, 1) * P->ng * 2))) return rc;
  double* tables = nullptr;
  if (!B.tasks.empty()) {
    FMM_HIP_TRY(hipMalloc(&tables, B.tasks.size() * (size_t)P->ng * sizeof(double)));
    const auto ts = std::chrono::steady_clock::now();
    if (sur && sur->kind == 1) {
      rc = gpu_table_tasks(P->medium, comps, smap, sur->d_lad, sur->dm, sur->tg, sur->d_tab, sur->nmax, B.tasks,
                           2 * p, tables, &P->stats.surrogate_tasks, st, nullptr);
    } else if (sur) {
      rc = gpu_surrogate_tables(P->medium, comps, smap, sur->d_lad, sur->dm, B.tasks, 2 * p, sur->net, tables,
                                &P->stats.surrogate_tasks, st, nullptr);
    } else {
      rc = gpu_sommerfeld_tables(P->medium, comps, B.tasks, 2 * p, tables, st);
    }
    P->stats.table_seconds = seconds_since(ts);
    if (rc == FMMLM_OK && sur) rc = surrogate_check(P, comps, B.tasks, tables, st);
    if (rc == FMMLM_OK && sur && !(P->stats.surrogate_check <= kSurrogateBound)) {
      // the learned or table form misses its bound on this plan's own tasks: the
      // quadrature serves every initial value and near-field kernel instead
      P->stats.surrogate_rejected = 1;
      P->stats.surrogate_tasks = 0;
      sur = nullptr;
      const auto tq = std::chrono::steady_clock::now();
      rc = gpu_sommerfeld_tables(P->medium, comps, B.tasks, 2 * p, tables, st);
      P->stats.table_seconds += seconds_since(tq);
    }
    if (rc) {
      hipFree(tables);
      return rc;
    }
  }
  rc = gpu_build_ops(P, B.free_off, B.reac_task, B.reac_phi, B.reac_S, tables, st);
  hipFree(tables);
  if (rc) return rc;
  if ((rc = dev_alloc(P, &P->Tfree, (size_t)std::max<int64_t>(P->nops, 1) * P->nrk * 32 * P->mrt))) return rc;
  if ((rc = gpu_build_real_ops(P, st))) return rc;
  if ((rc = dev_alloc(P, &P->Txl, (size_t)16 * P->nrk * 32 * P->mrt))) return rc;
  if ((rc = gpu_build_xlate_ops(P, st))) return rc;
  if (P->fp32) {
    const size_t nr = (size_t)(P->p + 1) * (P->p + 1);
    if ((rc = dev_alloc(P, &P->Tfree32, (size_t)std::max<int64_t>(P->nops, 1) * P->nrk * 32 * P->mrt))) return rc;
    // single-vector FP32 sources: rows padded to nrk (aligned, zero past nr)
    if (std::min(P->opts.max_rhs, 64) == 1 && (rc = dev_alloc(P, &P->M32, (size_t)P->NB * P->nrk))) return rc;
    (void)nr;
    if ((rc = dev_alloc(P, &P->qt32, P->NP))) return rc;
    if ((rc = dev_alloc(P, &P->pxh, P->NP)) || (rc = dev_alloc(P, &P->pxl, P->NP)) ||
        (rc = dev_alloc(P, &P->pyh, P->NP)) || (rc = dev_alloc(P, &P->pyl, P->NP)) ||
        (rc = dev_alloc(P, &P->phh, P->NP)) || (rc = dev_alloc(P, &P->phl, P->NP)))
      return rc;
    if ((rc = gpu_build_fp32(P, st))) return rc;
  }
  P->stats.n_free_ops = P->n_free_ops;
  P->stats.n_reaction_ops = (int64_t)B.reac_task.size();
  P->stats.n_sommerfeld_tasks = (int64_t)B.tasks.size();
  P->stats.ops_seconds = seconds_since(tphase);
  // ---- reaction near field values
  const int64_t npairs = (int64_t)rp_t.size();
  if ((rc = dev_alloc(P, &P->rp_val, (size_t)npairs))) return rc;
  if (npairs > 0) {
    int32_t *dt = nullptr, *ds = nullptr, *dc = nullptr;
    FMM_HIP_TRY(hipMalloc(&dt, npairs * 4));
    FMM_HIP_TRY(hipMalloc(&ds, npairs * 4));
    FMM_HIP_TRY(hipMalloc(&dc, npairs * 4));
    FMM_HIP_TRY(hipMemcpyAsync(dt, rp_t.data(), npairs * 4, hipMemcpyHostToDevice, st));
    FMM_HIP_TRY(hipMemcpyAsync(ds, rp_s.data(), npairs * 4, hipMemcpyHostToDevice, st));
    FMM_HIP_TRY(hipMemcpyAsync(dc, rp_c.data(), npairs * 4, hipMemcpyHostToDevice, st));
    const auto ts = std::chrono::steady_clock::now();
    if (sur && sur->kind == 1) {
      int64_t nfb = 0;
      rc = gpu_table_nearfield(P->medium, comps, smap, sur->d_lad, sur->dm, sur->tg, sur->d_tab, 2 * sur->nmax + 1,
                               dt, ds, dc, npairs, P->px, P->py, P->ph, P->rp_val, &nfb, st);
      P->stats.surrogate_pairs = npairs - nfb;
    } else if (sur) {
      int64_t nfb = 0;
      rc = gpu_surrogate_nearfield(P->medium, comps, smap, sur->d_lad, sur->dm, dt, ds, dc, npairs, P->px,
                                   P->py, P->ph, sur->net, P->rp_val, &nfb, st);
      P->stats.surrogate_pairs = npairs - nfb;
    } else {
      rc = gpu_reaction_nearfield(P->medium, comps, dt, ds, dc, npairs, P->px, P->py, P->ph, P->rp_val, st);
    }
    P->stats.nearfield_seconds = seconds_since(ts);
    hipFree(dt);
    hipFree(ds);
    hipFree(dc);
    if (rc) return rc;
    // the FP32 form's single-vector reaction P2P reads the values rounded to
    // FP32 (half the bytes of that HBM-bound stage; sums stay FP64)
    if (P->fp32) {
      if ((rc = dev_alloc(P, &P->rp_val32, (size_t)npairs))) return rc;
      if ((rc = gpu_round_f32(P->rp_val, npairs, P->rp_val32, st))) return rc;
    }
  }
  // ---- workspace (G = min(max_rhs, 64) vectors per pass)
  P->gmax = std::min(P->opts.max_rhs, 64);
  const size_t G = (size_t)P->gmax;
  const size_t nrr = (size_t)(P->p + 1) * (P->p + 1);
  if ((rc = dev_alloc(P, &P->qt, P->NP * G))) return rc;
  if ((rc = dev_alloc(P, &P->phit, P->NP * G))) return rc;
  if ((rc = dev_alloc(P, &P->phin, P->NP))) return rc;
  FMM_HIP_TRY(hipStreamCreateWithFlags(&P->s_near, hipStreamNonBlocking));
  FMM_HIP_TRY(hipStreamCreateWithFlags(&P->s_top, hipStreamNonBlocking));
  for (hipEvent_t* e : {&P->ev_q, &P->ev_m, &P->ev_near, &P->ev_top, &P->ev_l, &P->ev_done})
    FMM_HIP_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
  if ((rc = dev_alloc(P, &P->M, (size_t)P->NB * nrr * G))) return rc;
  if ((rc = dev_alloc(P, &P->Lx, (size_t)P->NB * nrr * G))) return rc;
  // FP32 sources of the batched form: [vector][box][nrk] (aligned rows, zero past nr)
  if (P->fp32 && G > 1 && (rc = dev_alloc(P, &P->M32, (size_t)P->NB * P->nrk * G))) return rc;
  if (P->fp32 && (rc = gpu_tune_m2l(P, st))) return rc;
  if (G > 1) {
    if ((rc = dev_alloc(P, &P->qb64, P->NP * 64))) return rc;
    if ((rc = dev_alloc(P, &P->qu, (size_t)P->N * 64))) return rc;
    if (P->fp32 && (rc = dev_alloc(P, &P->qb32, P->NP * 64))) return rc;
    std::vector<int32_t> bb;
    for (int64_t b = 0; b < P->NB; ++b)
      if (mptr[b + 1] > mptr[b]) {
        if (B.boxes[b].level < P->opts.fp64_top_levels) P->bbox_split = (int64_t)bb.size() + 1;
        bb.push_back((int32_t)b);
      }
    P->nbbox = (int64_t)bb.size();
    if ((rc = dev_upload(P, &P->bbox, bb, st))) return rc;
    if (P->fp32 && P->bbox_split > 0) {
      // the FP64 top levels of the batched FP32 form: work items of at most
      // kBatchTopItem entries of one box (few boxes, long entry lists)
      std::vector<int32_t> items, iptr(1, 0);
      for (int64_t bi = 0; bi < P->bbox_split; ++bi) {
        const int32_t b = bb[bi];
        for (int32_t e = mptr[b]; e < mptr[b + 1]; e += kBatchTopItem) {
          items.push_back((int32_t)bi);
          items.push_back(e);
          items.push_back(std::min<int32_t>(e + kBatchTopItem, mptr[b + 1]));
        }
        iptr.push_back((int32_t)(items.size() / 3));
      }
      P->n_btop_items = (int64_t)(items.size() / 3);
      if ((rc = dev_upload(P, &P->btop_items, items, st)) || (rc = dev_upload(P, &P->btop_iptr, iptr, st)))
        return rc;
      if ((rc = dev_alloc(P, &P->Pbtop, (size_t)std::max<int64_t>(P->n_btop_items, 1) * 64 * nrr)))
        return rc;
    }
    {
      auto octant = [&](int64_t b) {
        const HBox& bx = B.boxes[b];
        return (bx.ix & 1) | ((bx.iy & 1) << 1) | ((bx.ih & 1) << 2);
      };
      std::vector<int32_t> uptr(P->NB + 1, 0), usrc, uop, ub, dptr(P->NB + 1, 0), dsrc, dop, db;
      P->bu_lev.assign(1, 0);
      P->bd_lev.assign(1, 0);
      for (int l = 0; l <= P->maxlev; ++l) {
        for (int64_t b = P->lev_off[l]; b < P->lev_off[l + 1]; ++b) {
          const HBox& bx = B.boxes[b];
          if (bx.nchild > 0) ub.push_back((int32_t)b);
          if (l >= 1) db.push_back((int32_t)b);
        }
        P->bu_lev.push_back((int64_t)ub.size());
        P->bd_lev.push_back((int64_t)db.size());
      }
      for (int64_t b = 0; b < P->NB; ++b) {
        const HBox& bx = B.boxes[b];
        for (int k = 0; k < bx.nchild; ++k) {
          usrc.push_back(bx.child0 + k);
          uop.push_back(octant(bx.child0 + k));
        }
        uptr[b + 1] = (int32_t)usrc.size();
        if (bx.level >= 1) {
          dsrc.push_back(bx.parent);
          dop.push_back(8 + octant(b));
        }
        dptr[b + 1] = (int32_t)dsrc.size();
      }
      if ((rc = dev_upload(P, &P->bu_ptr, uptr, st)) || (rc = dev_upload(P, &P->bu_src, usrc, st)) ||
          (rc = dev_upload(P, &P->bu_op, uop, st)) || (rc = dev_upload(P, &P->bu_boxes, ub, st)) ||
          (rc = dev_upload(P, &P->bd_ptr, dptr, st)) || (rc = dev_upload(P, &P->bd_src, dsrc, st)) ||
          (rc = dev_upload(P, &P->bd_op, dop, st)) || (rc = dev_upload(P, &P->bd_boxes, db, st)))
        return rc;
    }
    if (P->fp32 && (rc = gpu_tune_batch(P, st))) return rc;
  }
  FMM_HIP_TRY(hipStreamSynchronize(st));
  if (P->fp32 && (rc = gpu_tune_eval(P, st))) return rc;
  FMM_HIP_TRY(hipStreamSynchronize(st));
  if ((rc = tune_batch_width(P, st))) return rc;
  return FMMLM_OK;
}

// Least squares min ||A x - b||_2 for a dense m x n matrix (row-major, m >= n)
// by Householder QR on unit-norm columns; x [n].  Returns false if a column
// is zero or the factor is singular.
bool lstsq_qr(std::vector<double> A, std::vector<double> b, int m, int n, std::vector<double>& x) {
  std::vector<double> cs(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double ss = 0.0;
    for (int i = 0; i < m; ++i) ss += A[(size_t)i * n + j] * A[(size_t)i * n + j];
    if (!(ss > 0.0)) return false;
    cs[j] = 1.0 / std::sqrt(ss);
    for (int i = 0; i < m; ++i) A[(size_t)i * n + j] *= cs[j];
  }
  for (int j = 0; j < n; ++j) {
    double nrm = 0.0;
    for (int i = j; i < m; ++i) nrm += A[(size_t)i * n + j] * A[(size_t)i * n + j];
    nrm = std::sqrt(nrm);
    if (!(nrm > 0.0)) return false;
    const double alpha = A[(size_t)j * n + j] > 0.0 ? -nrm : nrm;
    std::vector<double> v(m - j);
    for (int i = j; i < m; ++i) v[i - j] = A[(size_t)i * n + j];
    v[0] -= alpha;
    double vv = 0.0;
    for (double t : v) vv += t * t;
    if (vv > 0.0) {
      for (int c = j; c < n; ++c) {
        double dot = 0.0;
        for (int i = j; i < m; ++i) dot += v[i - j] * A[(size_t)i * n + c];
        const double f = 2.0 * dot / vv;
        for (int i = j; i < m; ++i) A[(size_t)i * n + c] -= f * v[i - j];
      }
      double dot = 0.0;
      for (int i = j; i < m; ++i) dot += v[i - j] * b[i];
      const double f = 2.0 * dot / vv;
      for (int i = j; i < m; ++i) b[i] -= f * v[i - j];
    }
  }
  x.assign(n, 0.0);
  for (int j = n - 1; j >= 0; --j) {
    double t = b[j];
    for (int c = j + 1; c < n; ++c) t -= A[(size_t)j * n + c] * x[c];
    const double r = A[(size_t)j * n + j];
    if (!(std::fabs(r) > 0.0)) return false;
    x[j] = t / r;
  }
  for (int j = 0; j < n; ++j) x[j] *= cs[j];
  return true;
}

// Ladder of each surrogate component: sigma(k) e^{k zinf} - sinf ~ sum_j c_j
// t^j, t = e^{-k delta}, j = 1..kLadder, fitted in least squares with the
// weight e^{-k zmin} (zmin = dmin / 10, the smallest height sum the fit is
// tuned for) on 200 uniform nodes in [0, 2.5 / dmin] and 300 geometric nodes
// up to kmax = min(500 / dmin, 600 / zinf).  The densities come from the GPU
// (the plan's own recursion); the fit runs once per surrogate on the host.
int fit_ladders(fmmlm_surrogate_s* S, hipStream_t st) {
  const double dmin = S->dm.dmin, delta = S->dm.delta, zmin = 0.1 * dmin;
  const int nlin = 200, ngeo = 300, m = nlin + ngeo;
  const size_t nc = S->comps.size();
  S->lad.assign(nc * kLadder, 0.0);
  S->ladder_fit = 0.0;
  std::vector<double> kre(m), kim(m, 0.0), ore(m), oim(m), A((size_t)m * kLadder), b(m), x;
  for (size_t c = 0; c < nc; ++c) {
    const CompInfo& ci = S->comps[c];
    double kmax = 500.0 / dmin;
    if (ci.zinf > 0.0) kmax = std::min(kmax, 600.0 / ci.zinf);
    const double k1 = std::min(2.5 / dmin, 0.5 * kmax);
    for (int i = 0; i < nlin; ++i) kre[i] = k1 * i / nlin;
    for (int i = 0; i < ngeo; ++i) kre[nlin + i] = k1 * std::pow(kmax / k1, (double)i / (ngeo - 1));
    int rc = gpu_density(S->medium, ci, m, kre.data(), kim.data(), ore.data(), oim.data(), st);
    if (rc) return rc;
    double gn = 0.0;
    for (int i = 0; i < m; ++i) {
      const double k = kre[i], w = std::exp(-k * zmin), t = std::exp(-k * delta);
      b[i] = w * (ore[i] * std::exp(k * ci.zinf) - ci.sinf);
      gn += b[i] * b[i];
      double tj = t;
      for (int j = 0; j < kLadder; ++j, tj *= t) A[(size_t)i * kLadder + j] = w * tj;
    }
    if (!(gn > 0.0)) continue;  // remainder identically zero: no rungs
    if (!lstsq_qr(A, b, m, kLadder, x)) {
      set_last_error("the ladder fit of a reaction density failed");
      return FMMLM_EUNSUPPORTED;
    }
    double rn = 0.0;
    for (int i = 0; i < m; ++i) {
      double f = 0.0;
      for (int j = 0; j < kLadder; ++j) f += A[(size_t)i * kLadder + j] * x[j];
      rn += (f - b[i]) * (f - b[i]);
    }
    S->ladder_fit = std::max(S->ladder_fit, std::sqrt(rn / gn));
    std::copy(x.begin(), x.end(), S->lad.begin() + c * kLadder);
  }
  FMM_HIP_TRY(hipMalloc(&S->d_lad, S->lad.size() * sizeof(double)));
  FMM_HIP_TRY(hipMemcpy(S->d_lad, S->lad.data(), S->lad.size() * sizeof(double), hipMemcpyHostToDevice));
  return FMMLM_OK;
}

// Output unit of the network: the rms of the targets over a pilot sample.
int pilot_yscale(fmmlm_surrogate_s* S, uint64_t seed, hipStream_t st) {
  constexpr int64_t kPilot = 32768;
  const int nout = 2 * S->nmax + 1;
  int32_t* dc = nullptr;
  float *df = nullptr, *dy = nullptr;
  S->dm.yscale = 1.0;
  int rc = FMMLM_OK;
  hipError_t e = hipMalloc(&dc, kPilot * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&df, kPilot * 4 * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&dy, (size_t)kPilot * nout * sizeof(float));
  if (e != hipSuccess) {
    set_last_error(hipGetErrorString(e));
    rc = FMMLM_EDEVICE;
  }
  std::vector<float> y((size_t)kPilot * nout);
  if (rc == FMMLM_OK)
    rc = gpu_surrogate_samples(S->medium, S->comps, S->d_lad, S->dm, S->nmax, seed ^ 0x51CA1Eull, kPilot, dc, df,
                               dy, st);
  if (rc == FMMLM_OK && (e = hipMemcpy(y.data(), dy, y.size() * sizeof(float), hipMemcpyDeviceToHost)) !=
                            hipSuccess) {
    set_last_error(hipGetErrorString(e));
    rc = FMMLM_EDEVICE;
  }
  hipFree(dc);
  hipFree(df);
  hipFree(dy);
  if (rc) return rc;
  double ss = 0.0;
  for (float v : y) ss += (double)v * v;
  const double rms = std::sqrt(ss / y.size());
  if (rms > 0.0 && std::isfinite(rms)) S->dm.yscale = rms;
  return FMMLM_OK;
}

}  // namespace
}  // namespace fmmlm

using namespace fmmlm;

extern "C" {

void fmmlm_default_opts(fmmlm_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->leaf_cap = 64;
  o->precision = FMMLM_FP64;
  o->fp64_top_levels = 3;
  o->max_rhs = 1;
  o->mac_d2 = 6;
}

}  // extern "C"

// The plan for the classic conditions (acoef null, eps the permittivities) or
// for the general ones (acoef = a on the host, eps = b / a).
static int plan_impl(int32_t n_interfaces, const double* z_interfaces, const double* eps, const double* acoef,
                     int64_t n, const double* x, const double* y, const double* z, const int32_t* layer_id,
                     int32_t p, const fmmlm_opts* opts, void* hip_stream, fmmlm_plan_t* out) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!out) return FMMLM_EINVAL;
  *out = nullptr;
  if (!z_interfaces || !eps || !x || !y || !z || !layer_id) return FMMLM_EINVAL;
  if (n < 1 || n >= ((int64_t)1 << 31) - 1) return FMMLM_EINVAL;
  if (p < 1 || p > FMMLM_PMAX) return FMMLM_EINVAL;
  if (n_interfaces < 1 || n_interfaces > kMaxL) return FMMLM_EINVAL;
  fmmlm_opts o;
  fmmlm_default_opts(&o);
  if (opts) o = *opts;
  if (o.leaf_cap < 1 || o.max_rhs < 1) return FMMLM_EINVAL;
  if (o.mac_d2 < 4 || o.mac_d2 > 12) return FMMLM_EINVAL;
  if (o.precision != FMMLM_FP64 && o.precision != FMMLM_FP32_COMPENSATED) return FMMLM_EINVAL;
  for (int i = 0; i < 2; ++i)
    if (o.reserved[i] != 0) return FMMLM_EINVAL;
  if (o.graph != 0 && o.graph != 1) return FMMLM_EINVAL;
  if (o.fp64_top_levels < 0 || o.fp64_top_levels > kMaxLevel + 1) return FMMLM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (o.surrogate) {
    // the network must describe this medium and cover orders up to 2p
    const fmmlm_surrogate_s* S = o.surrogate;
    if (S->L != n_interfaces || S->p < p) return FMMLM_EINVAL;
  }
  std::vector<double> dv, ev, X, Y, Z;
  std::vector<int32_t> LAY;
  int rc;
  if ((rc = fetch(z_interfaces, n_interfaces, dv))) return rc;
  if ((rc = fetch(eps, n_interfaces + 1, ev))) return rc;
  if ((rc = validate_medium(n_interfaces, dv, ev))) return rc;
  if (o.surrogate && (o.surrogate->d != dv || o.surrogate->eps != ev)) {
    set_last_error("the surrogate was trained for another medium");
    return FMMLM_EINVAL;
  }
  if (o.surrogate && acoef) {
    set_last_error("the learned form is built for the classic interface conditions");
    return FMMLM_EUNSUPPORTED;
  }
  if ((rc = fetch(x, n, X)) || (rc = fetch(y, n, Y)) || (rc = fetch(z, n, Z)) || (rc = fetch(layer_id, n, LAY)))
    return rc;
  const int L = n_interfaces;
  double ext = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(X[i]) || !std::isfinite(Y[i]) || !std::isfinite(Z[i])) return FMMLM_EINVAL;
    const int l = LAY[i];
    if (l < 0 || l > L) return FMMLM_ELAYER;
    if (l <= L - 1 && !(Z[i] >= dv[l])) return FMMLM_ELAYER;
    if (l >= 1 && !(Z[i] <= dv[l - 1])) return FMMLM_ELAYER;
    ext = std::max(ext, std::fabs(Z[i]));
  }
  fmmlm_plan_s* P = new (std::nothrow) fmmlm_plan_s();
  if (!P) return FMMLM_ENOMEM;
  std::memset(&P->stats, 0, sizeof(P->stats));
  P->L = L;
  P->d = dv;
  P->eps = ev;
  P->medium = make_medium(L, dv.data(), ev.data());
  if (acoef)
    for (int i = 0; i <= L; ++i) P->medium.acoef[i] = acoef[i];
  P->N = n;
  P->p = p;
  P->nc = ncoef(p);
  P->ng = ncoef(2 * p);
  P->opts = o;
  P->fp32 = (o.precision == FMMLM_FP32_COMPENSATED);
  try {
    rc = build_plan(P, X, Y, Z, LAY, st);
  } catch (const std::bad_alloc&) {
    rc = FMMLM_ENOMEM;
  }
  if (rc) {
    (void)hipStreamSynchronize(st);
    free_plan(P);
    return rc;
  }
  P->opts.surrogate = nullptr;  // not kept past planning
  P->stats.n_points = n;
  P->stats.n_tree_points = P->NP;
  P->stats.n_trees = (int32_t)P->trees.size();
  P->stats.p = p;
  P->stats.max_level = P->maxlev;
  P->stats.precision = o.precision;
  P->stats.n_boxes = P->NB;
  P->stats.n_leaves = P->nleaves;
  P->stats.root_side = P->W;
  P->stats.x0 = P->x0;
  P->stats.y0 = P->y0;
  P->stats.device_bytes = P->device_bytes;
  P->stats.plan_seconds = seconds_since(t0);
  *out = P;
  return FMMLM_OK;
}

extern "C" {

int fmm_layered_plan(int32_t n_interfaces, const double* z_interfaces, const double* eps, int64_t n,
                     const double* x, const double* y, const double* z, const int32_t* layer_id, int32_t p,
                     const fmmlm_opts* opts, void* hip_stream, fmmlm_plan_t* out) {
  return plan_impl(n_interfaces, z_interfaces, eps, nullptr, n, x, y, z, layer_id, p, opts, hip_stream, out);
}

int fmm_layered_plan_general(int32_t n_interfaces, const double* z_interfaces, const double* a, const double* b,
                             int64_t n, const double* x, const double* y, const double* z, const int32_t* layer_id,
                             int32_t p, const fmmlm_opts* opts, void* hip_stream, fmmlm_plan_t* out) {
  if (!out) return FMMLM_EINVAL;
  *out = nullptr;
  if (!a || !b || n_interfaces < 1 || n_interfaces > kMaxL) return FMMLM_EINVAL;
  std::vector<double> av, bv;
  int rc;
  if ((rc = fetch(a, n_interfaces + 1, av)) || (rc = fetch(b, n_interfaces + 1, bv))) return rc;
  std::vector<double> ev(n_interfaces + 1);
  for (int i = 0; i <= n_interfaces; ++i) {
    if (!std::isfinite(av[i]) || !(av[i] > 0.0) || !std::isfinite(bv[i]) || !(bv[i] > 0.0)) return FMMLM_EEPS;
    ev[i] = bv[i] / av[i];
  }
  return plan_impl(n_interfaces, z_interfaces, ev.data(), av.data(), n, x, y, z, layer_id, p, opts, hip_stream,
                   out);
}

}  // extern "C"

namespace fmmlm {

int plan_acquire(fmmlm_plan_s* P, hipStream_t st) {
  if (P->busy.exchange(1)) {
    set_last_error("another call is enqueuing work on the plan");
    return FMMLM_EBUSY;
  }
  if (P->done_recorded && st != P->done_stream) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const bool capturing = hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
    if (!capturing) {
      const hipError_t e = hipEventQuery(P->ev_done);
      (void)hipGetLastError();  // a pending event is not an error of the next call
      if (e == hipErrorNotReady) {
        P->busy.store(0);
        set_last_error("the plan's last evaluation, on another stream, has not finished");
        return FMMLM_EBUSY;
      }
    }
    (void)hipGetLastError();
  }
  return FMMLM_OK;
}

void plan_release(fmmlm_plan_s* P, hipStream_t st, bool record) {
  if (record && P->ev_done) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const bool capturing = hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
    (void)hipGetLastError();
    if (!capturing && hipEventRecord(P->ev_done, st) == hipSuccess) {
      P->done_stream = st;
      P->done_recorded = true;
    }
  }
  P->busy.store(0);
}

}  // namespace fmmlm

extern "C" {

int fmm_layered_eval(fmmlm_plan_t plan, int32_t nrhs, const double* q, int64_t ldq, double* phi, int64_t ldphi,
                     uint32_t parts, void* hip_stream) {
  if (!plan || !q || !phi) return FMMLM_EINVAL;
  if (nrhs < 1 || nrhs > plan->opts.max_rhs) return FMMLM_EINVAL;
  if (ldq < plan->N || ldphi < plan->N) return FMMLM_EINVAL;
  if (parts == 0 || (parts & ~(FMMLM_FREE | FMMLM_REACTION))) return FMMLM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int rc = plan_acquire(plan, st);
  if (rc) return rc;
  rc = fmmlm::eval_held(plan, nrhs, q, ldq, phi, ldphi, parts, st);
  plan_release(plan, st, rc == FMMLM_OK);
  return rc;
}

}  // extern "C"

// The evaluation proper, for a caller that holds the plan (plan_acquire) and
// has checked the arguments.
int fmmlm::eval_held(fmmlm_plan_t plan, int32_t nrhs, const double* q, int64_t ldq, double* phi, int64_t ldphi,
                     uint32_t parts, hipStream_t st) {
  auto launch = [&]() -> int {
    if (nrhs < plan->batch_min) {
      for (int r = 0; r < nrhs; ++r) {
        hipEvent_t* ev = nullptr;
        if (plan->prof_used < plan->prof_cap) ev = &plan->prof_ev[(size_t)plan->prof_used++ * (FMMLM_NSTAGES + 1)];
        if (int rc = gpu_eval_one(plan, q + (int64_t)r * ldq, phi + (int64_t)r * ldphi, parts, st, ev)) return rc;
      }
      return FMMLM_OK;
    }
    for (int r0 = 0; r0 < nrhs; r0 += plan->gmax) {
      const int g = std::min(plan->gmax, nrhs - r0);
      if (g < plan->batch_min) {
        // a narrow last pass: vector by vector
        for (int r = r0; r < r0 + g; ++r) {
          hipEvent_t* ev = nullptr;
          if (plan->prof_used < plan->prof_cap) ev = &plan->prof_ev[(size_t)plan->prof_used++ * (FMMLM_NSTAGES + 1)];
          if (int rc = gpu_eval_one(plan, q + (int64_t)r * ldq, phi + (int64_t)r * ldphi, parts, st, ev)) return rc;
        }
        continue;
      }
      hipEvent_t* ev = nullptr;
      if (plan->prof_used < plan->prof_cap) ev = &plan->prof_ev[(size_t)plan->prof_used++ * (FMMLM_NSTAGES + 1)];
      int rc = gpu_eval_batch(plan, g, q + (int64_t)r0 * ldq, ldq, phi + (int64_t)r0 * ldphi, ldphi, parts, st, ev);
      if (rc) return rc;
    }
    return FMMLM_OK;
  };
  const bool profiling = plan->prof_used < plan->prof_cap;
  if (!plan->opts.graph || st == nullptr || profiling) return launch();
  // graph mode: replay while the arguments are the same, capture anew otherwise
  const GraphKey key{nrhs, q, ldq, phi, ldphi, parts, st};
  if (plan->gexec && plan->gkey == key) {
    FMM_HIP_TRY(hipGraphLaunch(plan->gexec, st));
    return FMMLM_OK;
  }
  drop_graph(plan);
  FMM_HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  int rc = launch();
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(st, &g);
  if (rc == FMMLM_OK && e != hipSuccess) {
    set_last_error(hipGetErrorString(e));
    rc = FMMLM_EDEVICE;
  }
  if (rc == FMMLM_OK) {
    e = hipGraphInstantiate(&plan->gexec, g, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(plan->gexec, st);
    if (e != hipSuccess) {
      set_last_error(hipGetErrorString(e));
      rc = FMMLM_EDEVICE;
    }
  }
  if (g) (void)hipGraphDestroy(g);
  if (rc == FMMLM_OK) {
    plan->gkey = key;
  } else {
    drop_graph(plan);
  }
  return rc;
}

extern "C" {

int fmm_layered_plan_set_variants(fmmlm_plan_t plan, int32_t m2l_variant, int32_t batch_variant,
                                  int32_t batch_min_rhs) {
  if (!plan) return FMMLM_EINVAL;
  const int nm = plan->mrt == 4 ? kM2LVariants : 1;
  const int nb = plan->mrt == 4 ? 2 * kBatchShapes : 2;
  if (m2l_variant < -1 || m2l_variant >= nm || batch_variant < -1 || batch_variant >= nb) return FMMLM_EINVAL;
  if (batch_min_rhs != -1 && (batch_min_rhs < 2 || batch_min_rhs > 65)) return FMMLM_EINVAL;
  if (m2l_variant >= 0) plan->m2l_variant = plan->stats.m2l_variant = m2l_variant;
  if (batch_variant >= 0) plan->batch_variant = plan->stats.batch_variant = batch_variant;
  if (batch_min_rhs >= 0) plan->batch_min = plan->stats.batch_min_rhs = batch_min_rhs;
  drop_graph(plan);  // a captured evaluation holds the old launches
  return FMMLM_OK;
}

int fmm_layered_destroy(fmmlm_plan_t plan) {
  if (!plan) return FMMLM_OK;
  (void)hipDeviceSynchronize();
  free_plan(plan);
  return FMMLM_OK;
}

const char* fmm_layered_strerror(int code) {
  static thread_local std::string msg;
  const char* base = "unknown error";
  switch (code) {
    case FMMLM_OK: base = "success"; break;
    case FMMLM_EINVAL: base = "invalid argument"; break;
    case FMMLM_EINTERFACES: base = "interfaces must be finite and strictly decreasing"; break;
    case FMMLM_EEPS: base = "permittivities must be finite and positive"; break;
    case FMMLM_ELAYER: base = "layer id out of range or point outside its layer"; break;
    case FMMLM_EONINTERFACE: base = "point on an interface"; break;
    case FMMLM_EDEVICE: base = "HIP error"; break;
    case FMMLM_ENOMEM: base = "out of memory or list limit exceeded"; break;
    case FMMLM_EUNSUPPORTED: base = "unsupported option combination"; break;
    case FMMLM_EBUSY: base = "the plan is in use by another evaluation"; break;
    default: break;
  }
  msg = base;
  if (code == FMMLM_EDEVICE || code == FMMLM_ENOMEM || code == FMMLM_EBUSY) {
    if (!g_last_error.empty()) msg += ": " + g_last_error;
  }
  return msg.c_str();
}

int fmm_layered_plan_stats(fmmlm_plan_t plan, fmmlm_stats* out) {
  if (!plan || !out) return FMMLM_EINVAL;
  *out = plan->stats;
  return FMMLM_OK;
}

int fmm_layered_plan_tree(fmmlm_plan_t plan, int32_t t, int32_t* layer, int32_t* side, int64_t* n,
                          uint64_t* keys, int64_t* perm) {
  if (!plan || t < 0 || t >= (int32_t)plan->trees.size()) return FMMLM_EINVAL;
  const TreeInfo& T = plan->trees[t];
  if (layer) *layer = T.layer;
  if (side) *side = T.side;
  if (n) *n = T.n;
  if (keys) std::memcpy(keys, T.keys.data(), T.n * sizeof(uint64_t));
  if (perm) std::memcpy(perm, T.perm.data(), T.n * sizeof(int64_t));
  return FMMLM_OK;
}

int fmm_layered_plan_lists(fmmlm_plan_t plan, int32_t which, int64_t* count, int32_t* out) {
  if (!plan || !count || which < 0 || which > 3) return FMMLM_EINVAL;
  auto get = [](const int32_t* d, int64_t n, std::vector<int32_t>& h) -> int {
    h.assign((size_t)std::max<int64_t>(n, 0), 0);
    if (n > 0) FMM_HIP_TRY(hipMemcpy(h.data(), d, n * sizeof(int32_t), hipMemcpyDeviceToHost));
    return FMMLM_OK;
  };
  int rc;
  std::vector<int32_t> a, b, c, e;
  if (which == 0) {
    *count = plan->NB;
    if (!out) return FMMLM_OK;
    std::vector<int32_t> lev;
    if ((rc = get(plan->bstart, plan->NB, a)) || (rc = get(plan->bcount, plan->NB, b)) ||
        (rc = get(plan->bparent, plan->NB, c)) || (rc = get(plan->blevel, plan->NB, lev)))
      return rc;
    for (int64_t i = 0; i < plan->NB; ++i) {
      out[4 * i] = a[i];
      out[4 * i + 1] = b[i];
      out[4 * i + 2] = c[i];
      out[4 * i + 3] = lev[i];
    }
    return FMMLM_OK;
  }
  if (which == 1) {
    if ((rc = get(plan->m2l_ptr, plan->NB + 1, a))) return rc;
    *count = a[plan->NB];
    if (!out) return FMMLM_OK;
    if ((rc = get(plan->m2l_nfree, plan->NB, b)) || (rc = get(plan->m2l_src, a[plan->NB], c))) return rc;
    for (int64_t t = 0; t < plan->NB; ++t)
      for (int32_t k = a[t]; k < a[t + 1]; ++k) {
        out[3 * k] = (int32_t)t;
        out[3 * k + 1] = c[k];
        out[3 * k + 2] = (k - a[t] < b[t]) ? 1 : 0;
      }
    return FMMLM_OK;
  }
  const int32_t* ptr = (which == 2) ? plan->p2p_ptr : plan->rp_ptr;
  const int32_t* src = (which == 2) ? plan->p2p_src : plan->rp_src;
  if ((rc = get(ptr, plan->nleaves + 1, a))) return rc;
  *count = a[plan->nleaves];
  if (!out) return FMMLM_OK;
  if ((rc = get(plan->leaves, plan->nleaves, b)) || (rc = get(src, 2 * (int64_t)a[plan->nleaves], c))) return rc;
  for (int64_t li = 0; li < plan->nleaves; ++li)
    for (int32_t k = a[li]; k < a[li + 1]; ++k) {
      out[3 * k] = b[li];
      out[3 * k + 1] = c[2 * k];
      out[3 * k + 2] = c[2 * k + 1];
    }
  return FMMLM_OK;
}

int fmm_layered_sommerfeld(int32_t n_interfaces, const double* z_interfaces, const double* eps, int32_t lt,
                           int32_t ls, int32_t a, int32_t b, double S, int64_t npts, const double* rho,
                           const double* z, int32_t nmax, double* out, void* hip_stream) {
  if (npts < 1 || !rho || !z || !out || nmax < 0 || nmax > 2 * FMMLM_PMAX || !(S > 0.0)) return FMMLM_EINVAL;
  Medium md;
  std::memset(&md, 0, sizeof(md));
  if (n_interfaces > 0) {
    if (!z_interfaces || !eps) return FMMLM_EINVAL;
    std::vector<double> dv(z_interfaces, z_interfaces + n_interfaces), ev(eps, eps + n_interfaces + 1);
    int rc = validate_medium(n_interfaces, dv, ev);
    if (rc) return rc;
    md = make_medium(n_interfaces, dv.data(), ev.data());
    const int L = n_interfaces;
    if (lt < 0 || lt > L || ls < 0 || ls > L || a < 1 || a > 2 || b < 1 || b > 2) return FMMLM_EINVAL;
    if ((a == 1 && lt > L - 1) || (a == 2 && lt < 1) || (b == 1 && ls > L - 1) || (b == 2 && ls < 1))
      return FMMLM_EINVAL;
  }
  std::vector<CompInfo> comps(1);
  comps[0] = make_comp(md, lt, ls, a, b);
  std::vector<SommTask> tasks(npts);
  for (int64_t i = 0; i < npts; ++i) {
    if (!(rho[i] >= 0.0) || !(z[i] > 0.0)) return FMMLM_EINVAL;
    tasks[i] = SommTask{0, S, rho[i], z[i]};
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  double* d = nullptr;
  const size_t per = ncoef(nmax);
  FMM_HIP_TRY(hipMalloc(&d, npts * per * sizeof(double)));
  int rc = gpu_sommerfeld_tables(md, comps, tasks, nmax, d, st);
  if (rc == FMMLM_OK) {
    hipError_t e = hipMemcpy(out, d, npts * per * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      set_last_error(hipGetErrorString(e));
      rc = FMMLM_EDEVICE;
    }
  }
  hipFree(d);
  return rc;
}

int fmm_layered_sommerfeld_noalloc(int32_t n_interfaces, const double* z_interfaces, const double* eps,
                                   int32_t lt, int32_t ls, int32_t a, int32_t b, double S, int64_t npts,
                                   const double* rho, const double* z, int32_t nmax, double* out,
                                   void* hip_stream) {
  if (!rho || !z || !out || nmax < 0 || nmax > 2 * FMMLM_PMAX || !(S > 0.0) || !std::isfinite(S))
    return FMMLM_EINVAL;
  if (npts < 1 || npts > FMMLM_NOALLOC_MAX_POINTS) {
    set_last_error("fmm_layered_sommerfeld_noalloc: npts must be 1.." +
                   std::to_string(FMMLM_NOALLOC_MAX_POINTS));
    return FMMLM_EINVAL;
  }
  // the medium is read from fixed-size host arrays (no vectors: nothing is allocated)
  Medium md;
  std::memset(&md, 0, sizeof(md));
  if (n_interfaces < 0 || n_interfaces > kMaxL) return FMMLM_EINVAL;
  if (n_interfaces > 0) {
    if (!z_interfaces || !eps) return FMMLM_EINVAL;
    const int L = n_interfaces;
    for (int i = 0; i < L; ++i)
      if (!std::isfinite(z_interfaces[i]) || (i > 0 && !(z_interfaces[i] < z_interfaces[i - 1])))
        return FMMLM_EINTERFACES;
    for (int i = 0; i <= L; ++i)
      if (!std::isfinite(eps[i]) || !(eps[i] > 0.0)) return FMMLM_EEPS;
    md = make_medium(L, z_interfaces, eps);
    if (lt < 0 || lt > L || ls < 0 || ls > L || a < 1 || a > 2 || b < 1 || b > 2) return FMMLM_EINVAL;
    if ((a == 1 && lt > L - 1) || (a == 2 && lt < 1) || (b == 1 && ls > L - 1) || (b == 2 && ls < 1))
      return FMMLM_EINVAL;
  }
  const CompInfo c = make_comp(md, lt, ls, a, b);
  return gpu_sommerfeld_noalloc(md, c, S, npts, rho, z, nmax, out, static_cast<hipStream_t>(hip_stream));
}

int fmm_layered_density(int32_t n_interfaces, const double* z_interfaces, const double* eps, int32_t lt,
                        int32_t ls, int32_t a, int32_t b, int64_t nk, const double* k_re, const double* k_im,
                        double* out_re, double* out_im, void* hip_stream) {
  if (nk < 1 || !k_re || !k_im || !out_re || !out_im || !z_interfaces || !eps) return FMMLM_EINVAL;
  std::vector<double> dv(z_interfaces, z_interfaces + n_interfaces), ev(eps, eps + n_interfaces + 1);
  int rc = validate_medium(n_interfaces, dv, ev);
  if (rc) return rc;
  const int L = n_interfaces;
  if (lt < 0 || lt > L || ls < 0 || ls > L || a < 1 || a > 2 || b < 1 || b > 2) return FMMLM_EINVAL;
  if ((a == 1 && lt > L - 1) || (a == 2 && lt < 1) || (b == 1 && ls > L - 1) || (b == 2 && ls < 1))
    return FMMLM_EINVAL;
  Medium md = make_medium(L, dv.data(), ev.data());
  CompInfo c{lt, ls, a, b, 0.0, 0.0};
  return gpu_density(md, c, nk, k_re, k_im, out_re, out_im, static_cast<hipStream_t>(hip_stream));
}

int fmm_layered_density_asymptotic(int32_t n_interfaces, const double* z_interfaces, const double* eps,
                                   int32_t lt, int32_t ls, int32_t a, int32_t b, double* sinf,
                                   double* zinf) {
  if (!sinf || !zinf || !z_interfaces || !eps || n_interfaces < 1) return FMMLM_EINVAL;
  std::vector<double> dv(z_interfaces, z_interfaces + n_interfaces), ev(eps, eps + n_interfaces + 1);
  int rc = validate_medium(n_interfaces, dv, ev);
  if (rc) return rc;
  const int L = n_interfaces;
  if (lt < 0 || lt > L || ls < 0 || ls > L || a < 1 || a > 2 || b < 1 || b > 2) return FMMLM_EINVAL;
  if ((a == 1 && lt > L - 1) || (a == 2 && lt < 1) || (b == 1 && ls > L - 1) || (b == 2 && ls < 1))
    return FMMLM_EINVAL;
  Medium md = make_medium(L, dv.data(), ev.data());
  const CompInfo c = make_comp(md, lt, ls, a, b);
  *sinf = c.sinf;
  *zinf = c.zinf;
  return FMMLM_OK;
}

int fmm_layered_profile_begin(fmmlm_plan_t plan, int32_t max_evals) {
  if (!plan || max_evals < 1 || max_evals > 100000) return FMMLM_EINVAL;
  for (auto e : plan->prof_ev) (void)hipEventDestroy(e);
  plan->prof_ev.assign((size_t)max_evals * (FMMLM_NSTAGES + 1), nullptr);
  for (auto& e : plan->prof_ev) FMM_HIP_TRY(hipEventCreate(&e));
  plan->prof_cap = max_evals;
  plan->prof_used = 0;
  return FMMLM_OK;
}

int fmm_layered_profile_end(fmmlm_plan_t plan, double* stage_ms, int64_t* n_evals) {
  if (!plan || !stage_ms || !n_evals) return FMMLM_EINVAL;
  FMM_HIP_TRY(hipDeviceSynchronize());
  for (int s = 0; s < FMMLM_NSTAGES; ++s) stage_ms[s] = 0.0;
  for (int i = 0; i < plan->prof_used; ++i) {
    hipEvent_t* ev = &plan->prof_ev[(size_t)i * (FMMLM_NSTAGES + 1)];
    for (int s = 0; s < FMMLM_NSTAGES; ++s) {
      float ms = 0.f;
      FMM_HIP_TRY(hipEventElapsedTime(&ms, ev[s], ev[s + 1]));
      stage_ms[s] += ms;
    }
  }
  *n_evals = plan->prof_used;
  for (auto e : plan->prof_ev) (void)hipEventDestroy(e);
  plan->prof_ev.clear();
  plan->prof_cap = plan->prof_used = 0;
  return FMMLM_OK;
}

// ---- learned form ---------------------------------------------------------
void fmmlm_default_train_opts(fmmlm_train_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->nsamples = (int64_t)1 << 21;
  o->steps = 6000;
  o->batch = 8192;
  o->lr = 2e-3;
  o->seed = 1;
}

int fmm_layered_surrogate_create(int32_t n_interfaces, const double* z_interfaces, const double* eps, int32_t p,
                                 double rho_max, double zeta_max, uint64_t seed, fmmlm_surrogate_t* out) {
  if (!out) return FMMLM_EINVAL;
  *out = nullptr;
  if (!z_interfaces || !eps || p < 1 || p > FMMLM_PMAX) return FMMLM_EINVAL;
  if (!(rho_max > 0.0) || !(zeta_max > 0.0) || !std::isfinite(rho_max) || !std::isfinite(zeta_max))
    return FMMLM_EINVAL;
  if (n_interfaces < 1 || n_interfaces > kMaxL) return FMMLM_EINVAL;
  std::vector<double> dv, ev;
  int rc;
  if ((rc = fetch(z_interfaces, n_interfaces, dv))) return rc;
  if ((rc = fetch(eps, n_interfaces + 1, ev))) return rc;
  if ((rc = validate_medium(n_interfaces, dv, ev))) return rc;
  if (n_interfaces < 2) {
    set_last_error("the learned form needs at least two interfaces");
    return FMMLM_EUNSUPPORTED;
  }
  fmmlm_surrogate_s* S = new (std::nothrow) fmmlm_surrogate_s();
  if (!S) return FMMLM_ENOMEM;
  const int L = n_interfaces;
  S->L = L;
  S->d = dv;
  S->eps = ev;
  S->medium = make_medium(L, dv.data(), ev.data());
  S->p = p;
  S->nmax = 2 * p;
  double dmin = 0.0;
  for (int i = 1; i < L; ++i) {
    const double t = dv[i - 1] - dv[i];
    if (dmin == 0.0 || t < dmin) dmin = t;
  }
  S->dm = SurrogateDomain{rho_max, zeta_max, dmin, 2.0 * dmin, 1.0};
  std::vector<std::pair<int, int>> sides;
  for (int l = 0; l <= L; ++l)
    for (int side = 1; side <= 2; ++side) {
      if ((side == 1 && l > L - 1) || (side == 2 && l < 1)) continue;
      sides.push_back({l, side});
    }
  for (auto& t : sides)
    for (auto& u : sides) S->comps.push_back(make_comp(S->medium, t.first, u.first, t.second, u.second));
  S->net.ncomp = (int)S->comps.size();
  S->net.nout = 2 * S->nmax + 1;
  mlp_layout(S->net);
  (void)hipGetDevice(&S->device);
  hipStream_t st = nullptr;
  hipError_t e = hipMalloc(&S->net.params, S->net.nparams * sizeof(float));
  if (e != hipSuccess) {
    set_last_error(hipGetErrorString(e));
    rc = FMMLM_EDEVICE;
  }
  if (rc == FMMLM_OK) rc = fit_ladders(S, st);
  if (rc == FMMLM_OK) rc = pilot_yscale(S, seed, st);
  if (rc == FMMLM_OK) rc = gpu_mlp_init(S->net, seed, st);
  if (rc == FMMLM_OK && hipDeviceSynchronize() != hipSuccess) rc = FMMLM_EDEVICE;
  if (rc) {
    hipFree(S->net.params);
    hipFree(S->d_lad);
    delete S;
    return rc;
  }
  *out = S;
  return FMMLM_OK;
}

int fmm_layered_surrogate_create_for_plan(fmmlm_plan_t plan, uint64_t seed, fmmlm_surrogate_t* out) {
  if (!plan || !out) return FMMLM_EINVAL;
  return fmm_layered_surrogate_create(plan->L, plan->d.data(), plan->eps.data(), plan->p, std::sqrt(2.0) * plan->W,
                                      2.0 * plan->W, seed, out);
}

int fmm_layered_tables_create(int32_t n_interfaces, const double* z_interfaces, const double* eps, int32_t p,
                              double rho_max, double zeta_max, void* hip_stream, fmmlm_surrogate_t* out) {
  if (!out) return FMMLM_EINVAL;
  *out = nullptr;
  if (!z_interfaces || !eps || p < 1 || p > FMMLM_PMAX) return FMMLM_EINVAL;
  if (!(rho_max > 0.0) || !(zeta_max > 0.0) || !std::isfinite(rho_max) || !std::isfinite(zeta_max))
    return FMMLM_EINVAL;
  if (n_interfaces < 1 || n_interfaces > kMaxL) return FMMLM_EINVAL;
  std::vector<double> dv, ev;
  int rc;
  if ((rc = fetch(z_interfaces, n_interfaces, dv))) return rc;
  if ((rc = fetch(eps, n_interfaces + 1, ev))) return rc;
  if ((rc = validate_medium(n_interfaces, dv, ev))) return rc;
  if (n_interfaces < 2) {
    set_last_error("the table form needs at least two interfaces");
    return FMMLM_EUNSUPPORTED;
  }
  const auto t0 = std::chrono::steady_clock::now();
  fmmlm_surrogate_s* S = new (std::nothrow) fmmlm_surrogate_s();
  if (!S) return FMMLM_ENOMEM;
  const int L = n_interfaces;
  S->kind = 1;
  S->L = L;
  S->d = dv;
  S->eps = ev;
  S->medium = make_medium(L, dv.data(), ev.data());
  S->p = p;
  S->nmax = 2 * p;
  double dmin = 0.0;
  for (int i = 1; i < L; ++i) {
    const double t = dv[i - 1] - dv[i];
    if (dmin == 0.0 || t < dmin) dmin = t;
  }
  // values in the remainder's own unit (yscale 1)
  S->dm = SurrogateDomain{rho_max, zeta_max, dmin, 2.0 * dmin, 1.0};
  std::vector<std::pair<int, int>> sides;
  for (int l = 0; l <= L; ++l)
    for (int side = 1; side <= 2; ++side) {
      if ((side == 1 && l > L - 1) || (side == 2 && l < 1)) continue;
      sides.push_back({l, side});
    }
  for (auto& t : sides)
    for (auto& u : sides) S->comps.push_back(make_comp(S->medium, t.first, u.first, t.second, u.second));
  // panels no wider than the thinnest layer: the remainder's nearest singularity
  // (the first image beyond the leading one) lies at least 2 dmin off the real
  // (rho, zeta) domain, so each panel's Chebyshev interpolant converges fast
  auto panels = [&](double ext) {
    const int n = (int)std::ceil(ext / dmin - 1e-9);
    return std::min(std::max(n, 4), 48);
  };
  S->tg.npr = panels(rho_max);
  S->tg.npz = panels(zeta_max);
  S->tg.hr = rho_max / S->tg.npr;
  S->tg.hz = zeta_max / S->tg.npz;
  (void)hipGetDevice(&S->device);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int nout = 2 * S->nmax + 1;
  const size_t nval = S->comps.size() * (size_t)S->tg.npr * S->tg.npz * nout * kTabK * kTabK;
  hipError_t e = hipMalloc(&S->d_tab, nval * sizeof(double));
  if (e != hipSuccess) {
    set_last_error(hipGetErrorString(e));
    rc = FMMLM_ENOMEM;
  }
  if (rc == FMMLM_OK) rc = fit_ladders(S, st);
  if (rc == FMMLM_OK) rc = gpu_table_fill(S->medium, S->comps, S->d_lad, S->dm, S->tg, S->nmax, S->d_tab, st);
  if (rc) {
    hipFree(S->d_tab);
    hipFree(S->d_lad);
    delete S;
    return rc;
  }
  S->fill_seconds = seconds_since(t0);
  *out = S;
  return FMMLM_OK;
}

int fmm_layered_tables_create_for_plan(fmmlm_plan_t plan, void* hip_stream, fmmlm_surrogate_t* out) {
  if (!plan || !out) return FMMLM_EINVAL;
  return fmm_layered_tables_create(plan->L, plan->d.data(), plan->eps.data(), plan->p, std::sqrt(2.0) * plan->W,
                                   2.0 * plan->W, hip_stream, out);
}

int fmm_layered_tables_info(fmmlm_surrogate_t s, int32_t* npr, int32_t* npz, int64_t* bytes, double* seconds) {
  if (!s || s->kind != 1) return FMMLM_EINVAL;
  if (npr) *npr = s->tg.npr;
  if (npz) *npz = s->tg.npz;
  if (bytes)
    *bytes = (int64_t)(s->comps.size() * (size_t)s->tg.npr * s->tg.npz * (2 * s->nmax + 1) * kTabK * kTabK *
                       sizeof(double));
  if (seconds) *seconds = s->fill_seconds;
  return FMMLM_OK;
}

int fmm_layered_interp2d(int32_t npr, int32_t npz, double rho_max, double zeta_max, int32_t nout,
                         const double* nodes, int64_t npts, const double* rho, const double* zeta, double* out,
                         void* hip_stream) {
  if (npr < 1 || npz < 1 || npr > 4096 || npz > 4096 || nout < 1 || nout > 1024 || !nodes || npts < 1 || !rho ||
      !zeta || !out || !(rho_max > 0.0) || !(zeta_max > 0.0))
    return FMMLM_EINVAL;
  for (int64_t i = 0; i < npts; ++i)
    if (!(rho[i] >= 0.0 && rho[i] <= rho_max && zeta[i] >= 0.0 && zeta[i] <= zeta_max)) return FMMLM_EINVAL;
  TableGrid g;
  g.npr = npr;
  g.npz = npz;
  g.hr = rho_max / npr;
  g.hz = zeta_max / npz;
  const size_t nn = (size_t)npr * npz * nout * kTabK * kTabK;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  double *dn = nullptr, *dp = nullptr;
  FMM_HIP_TRY(hipMalloc(&dn, nn * sizeof(double)));
  if (hipMalloc(&dp, (size_t)npts * (2 + nout) * sizeof(double)) != hipSuccess) {
    hipFree(dn);
    set_last_error("fmm_layered_interp2d: allocation failed");
    return FMMLM_ENOMEM;
  }
  int rc = FMMLM_OK;
  hipError_t e = hipMemcpy(dn, nodes, nn * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dp, rho, npts * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dp + npts, zeta, npts * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    set_last_error(hipGetErrorString(e));
    rc = FMMLM_EDEVICE;
  }
  if (rc == FMMLM_OK) rc = gpu_interp2d(g, nout, dn, npts, dp, dp + npts, dp + 2 * npts, st);
  if (rc == FMMLM_OK && hipStreamSynchronize(st) != hipSuccess) rc = FMMLM_EDEVICE;
  if (rc == FMMLM_OK) {
    e = hipMemcpy(out, dp + 2 * npts, (size_t)npts * nout * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      set_last_error(hipGetErrorString(e));
      rc = FMMLM_EDEVICE;
    }
  }
  hipFree(dn);
  hipFree(dp);
  return rc;
}

int fmm_layered_surrogate_destroy(fmmlm_surrogate_t s) {
  if (!s) return FMMLM_EINVAL;
  hipFree(s->net.params);
  hipFree(s->d_lad);
  hipFree(s->d_tab);
  delete s;
  return FMMLM_OK;
}

int fmm_layered_surrogate_train(fmmlm_surrogate_t s, const fmmlm_train_opts* opts, void* hip_stream,
                                fmmlm_train_report* rep) {
  if (s && s->kind != 0) return FMMLM_EUNSUPPORTED;  // a table form has no network
  if (!s) return FMMLM_EINVAL;
  fmmlm_train_opts o;
  fmmlm_default_train_opts(&o);
  if (opts) o = *opts;
  for (int i = 0; i < 4; ++i)
    if (o.reserved[i] != 0) return FMMLM_EINVAL;
  if (o.nsamples < 128 || o.nsamples > ((int64_t)1 << 28) || o.steps < 0 || o.batch < 64 || o.batch % 64 ||
      o.batch > (1 << 20) || !(o.lr > 0.0))
    return FMMLM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int64_t n = o.nsamples, nval = n / 32, ntrain = n - nval;
  const int nout = s->net.nout;
  int32_t* comp = nullptr;
  float *feat = nullptr, *y = nullptr, *vout = nullptr;
  auto cleanup = [&]() {
    hipFree(comp);
    hipFree(feat);
    hipFree(y);
    hipFree(vout);
  };
  FMM_HIP_TRY(hipMalloc(&comp, n * sizeof(int32_t)));
  FMM_HIP_TRY(hipMalloc(&feat, n * 4 * sizeof(float)));
  FMM_HIP_TRY(hipMalloc(&y, (size_t)n * nout * sizeof(float)));
  FMM_HIP_TRY(hipMalloc(&vout, (size_t)std::max<int64_t>(nval, 1) * nout * sizeof(float)));
  fmmlm_train_report r;
  std::memset(&r, 0, sizeof(r));
  auto t0 = std::chrono::steady_clock::now();
  int rc = gpu_surrogate_samples(s->medium, s->comps, s->d_lad, s->dm, s->nmax, o.seed, n, comp, feat, y, st);
  r.sample_seconds = seconds_since(t0);
  if (rc == FMMLM_OK) {
    t0 = std::chrono::steady_clock::now();
    rc = gpu_mlp_train(s->net, comp, feat, y, ntrain, o.steps, o.batch, o.lr, o.seed, &r.loss_first,
                       &r.loss_last, st);
    r.train_seconds = seconds_since(t0);
  }
  if (rc == FMMLM_OK && nval > 0) {
    rc = gpu_mlp_forward(s->net, comp + ntrain, feat + ntrain * 4, nval, vout, nout, nout, nullptr, nullptr,
                         nullptr, st);
    std::vector<float> a((size_t)nval * nout), b((size_t)nval * nout);
    if (rc == FMMLM_OK) {
      hipError_t e = hipMemcpyAsync(a.data(), vout, a.size() * sizeof(float), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(b.data(), y + ntrain * nout, b.size() * sizeof(float), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        set_last_error(hipGetErrorString(e));
        rc = FMMLM_EDEVICE;
      }
    }
    double ss = 0.0, mx = 0.0;
    for (size_t i = 0; i < a.size(); ++i) {
      const double dd = (double)a[i] - (double)b[i];
      ss += dd * dd;
      mx = std::max(mx, std::fabs(dd));
    }
    r.val_rms = std::sqrt(ss / std::max<size_t>(a.size(), 1));
    r.val_max = mx;
  }
  cleanup();
  r.n_train = ntrain;
  r.n_val = nval;
  r.n_params = s->net.nparams;
  r.n_components = s->net.ncomp;
  r.n_outputs = nout;
  r.yscale = s->dm.yscale;
  r.ladder_fit = s->ladder_fit;
  if (rep) *rep = r;
  return rc;
}

int fmm_layered_surrogate_params(fmmlm_surrogate_t s, float* get, const float* set, int64_t* n) {
  if (s && s->kind != 0) return FMMLM_EUNSUPPORTED;  // a table form has no network
  if (!s) return FMMLM_EINVAL;
  if (n) *n = s->net.nparams;
  if (get) FMM_HIP_TRY(hipMemcpy(get, s->net.params, s->net.nparams * sizeof(float), hipMemcpyDeviceToHost));
  if (set) FMM_HIP_TRY(hipMemcpy(s->net.params, set, s->net.nparams * sizeof(float), hipMemcpyHostToDevice));
  return FMMLM_OK;
}

int fmm_layered_surrogate_grad(fmmlm_surrogate_t s, int64_t n, const int32_t* comp, const float* feat,
                               const float* target, double* loss, float* grad, void* hip_stream) {
  if (s && s->kind != 0) return FMMLM_EUNSUPPORTED;  // a table form has no network
  if (!s || n < 1 || n > ((int64_t)1 << 24) || !comp || !feat || !target || !loss || !grad) return FMMLM_EINVAL;
  for (int64_t i = 0; i < n; ++i)
    if (comp[i] < 0 || comp[i] >= s->net.ncomp) return FMMLM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int nout = s->net.nout;
  int32_t* dc = nullptr;
  float *df = nullptr, *dy = nullptr, *dg = nullptr;
  FMM_HIP_TRY(hipMalloc(&dc, n * sizeof(int32_t)));
  FMM_HIP_TRY(hipMalloc(&df, n * 4 * sizeof(float)));
  FMM_HIP_TRY(hipMalloc(&dy, (size_t)n * nout * sizeof(float)));
  FMM_HIP_TRY(hipMalloc(&dg, s->net.nparams * sizeof(float)));
  int rc = FMMLM_OK;
  hipError_t e = hipMemcpy(dc, comp, n * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(df, feat, n * 4 * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dy, target, (size_t)n * nout * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    set_last_error(hipGetErrorString(e));
    rc = FMMLM_EDEVICE;
  }
  if (rc == FMMLM_OK) rc = gpu_mlp_grad(s->net, dc, df, dy, n, dg, loss, st);
  if (rc == FMMLM_OK) {
    e = hipMemcpy(grad, dg, s->net.nparams * sizeof(float), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      set_last_error(hipGetErrorString(e));
      rc = FMMLM_EDEVICE;
    }
  }
  hipFree(dc);
  hipFree(df);
  hipFree(dy);
  hipFree(dg);
  return rc;
}

int fmm_layered_surrogate_forward(fmmlm_surrogate_t s, int64_t n, const int32_t* comp, const float* feat,
                                  float* out, void* hip_stream) {
  if (s && s->kind != 0) return FMMLM_EUNSUPPORTED;  // a table form has no network
  if (!s || n < 1 || n > ((int64_t)1 << 24) || !comp || !feat || !out) return FMMLM_EINVAL;
  for (int64_t i = 0; i < n; ++i)
    if (comp[i] < 0 || comp[i] >= s->net.ncomp) return FMMLM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int nout = s->net.nout;
  int32_t* dc = nullptr;
  float *df = nullptr, *dy = nullptr;
  FMM_HIP_TRY(hipMalloc(&dc, n * sizeof(int32_t)));
  if (hipMalloc(&df, n * 4 * sizeof(float)) != hipSuccess || hipMalloc(&dy, (size_t)n * nout * sizeof(float)) != hipSuccess) {
    hipFree(dc);
    hipFree(df);
    set_last_error("fmm_layered_surrogate_forward: allocation failed");
    return FMMLM_ENOMEM;
  }
  int rc = FMMLM_OK;
  hipError_t e = hipMemcpy(dc, comp, n * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(df, feat, n * 4 * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    set_last_error(hipGetErrorString(e));
    rc = FMMLM_EDEVICE;
  }
  if (rc == FMMLM_OK) rc = gpu_mlp_forward(s->net, dc, df, n, dy, nout, nout, nullptr, nullptr, nullptr, st);
  if (rc == FMMLM_OK) {
    e = hipMemcpy(out, dy, (size_t)n * nout * sizeof(float), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      set_last_error(hipGetErrorString(e));
      rc = FMMLM_EDEVICE;
    }
  }
  hipFree(dc);
  hipFree(df);
  hipFree(dy);
  return rc;
}

int fmm_layered_surrogate_adam(fmmlm_surrogate_t s, int32_t nsteps, const float* grads, const double* lr,
                               float* params_out, void* hip_stream) {
  if (s && s->kind != 0) return FMMLM_EUNSUPPORTED;  // a table form has no network
  if (!s || nsteps < 1 || nsteps > 64 || !grads || !lr) return FMMLM_EINVAL;
  for (int t = 0; t < nsteps; ++t)
    if (!std::isfinite(lr[t]) || !(lr[t] > 0.0)) return FMMLM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const size_t bytes = (size_t)nsteps * s->net.nparams * sizeof(float);
  float *dg = nullptr, *dt = nullptr;
  FMM_HIP_TRY(hipMalloc(&dg, bytes));
  if (hipMalloc(&dt, bytes) != hipSuccess) {
    hipFree(dg);
    set_last_error("fmm_layered_surrogate_adam: allocation failed");
    return FMMLM_ENOMEM;
  }
  int rc = FMMLM_OK;
  hipError_t e = hipMemcpy(dg, grads, bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    set_last_error(hipGetErrorString(e));
    rc = FMMLM_EDEVICE;
  }
  if (rc == FMMLM_OK) rc = gpu_mlp_adam_steps(s->net, nsteps, dg, lr, dt, st);
  if (rc == FMMLM_OK && params_out) {
    e = hipMemcpy(params_out, dt, bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      set_last_error(hipGetErrorString(e));
      rc = FMMLM_EDEVICE;
    }
  }
  hipFree(dg);
  hipFree(dt);
  return rc;
}

int fmm_layered_surrogate_samples(fmmlm_surrogate_t s, int64_t n, uint64_t seed, int32_t* comp, double* rho,
                                  double* zeta, float* feat, float* target, void* hip_stream) {
  if (s && s->kind != 0) return FMMLM_EUNSUPPORTED;  // a table form has no network
  if (!s || n < 1 || n > ((int64_t)1 << 24) || !comp || !rho || !zeta || !feat || !target) return FMMLM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int nout = s->net.nout;
  int32_t* dc = nullptr;
  float *df = nullptr, *dy = nullptr;
  double* drz = nullptr;
  FMM_HIP_TRY(hipMalloc(&dc, n * sizeof(int32_t)));
  FMM_HIP_TRY(hipMalloc(&df, n * 4 * sizeof(float)));
  FMM_HIP_TRY(hipMalloc(&dy, (size_t)n * nout * sizeof(float)));
  FMM_HIP_TRY(hipMalloc(&drz, n * 2 * sizeof(double)));
  int rc = gpu_surrogate_samples(s->medium, s->comps, s->d_lad, s->dm, s->nmax, seed, n, dc, df, dy, st, drz);
  std::vector<double> rz(2 * n);
  if (rc == FMMLM_OK) {
    hipError_t e = hipMemcpy(comp, dc, n * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(feat, df, n * 4 * sizeof(float), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(target, dy, (size_t)n * nout * sizeof(float), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(rz.data(), drz, n * 2 * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      set_last_error(hipGetErrorString(e));
      rc = FMMLM_EDEVICE;
    }
    for (int64_t i = 0; i < n; ++i) {
      rho[i] = rz[2 * i];
      zeta[i] = rz[2 * i + 1];
    }
  }
  hipFree(dc);
  hipFree(df);
  hipFree(dy);
  hipFree(drz);
  return rc;
}

int fmm_layered_surrogate_eval(fmmlm_surrogate_t s, int32_t lt, int32_t ls, int32_t a, int32_t b, double S,
                               int64_t npts, const double* rho, const double* z, int32_t nmax, double* out,
                               int32_t* used, void* hip_stream) {
  if (!s || npts < 1 || npts > ((int64_t)1 << 28) || !rho || !z || !out || nmax < 0 || nmax > s->nmax ||
      !(S > 0.0))
    return FMMLM_EINVAL;
  const int L = s->L;
  if (lt < 0 || lt > L || ls < 0 || ls > L || a < 1 || a > 2 || b < 1 || b > 2) return FMMLM_EINVAL;
  if ((a == 1 && lt > L - 1) || (a == 2 && lt < 1) || (b == 1 && ls > L - 1) || (b == 2 && ls < 1))
    return FMMLM_EINVAL;
  std::vector<CompInfo> comps{make_comp(s->medium, lt, ls, a, b)};
  std::vector<int32_t> smap{side_index(L, lt, a) * 2 * L + side_index(L, ls, b)};
  std::vector<SommTask> tasks(npts);
  for (int64_t i = 0; i < npts; ++i) {
    if (!(rho[i] >= 0.0) || !(z[i] > 0.0)) return FMMLM_EINVAL;
    tasks[i] = SommTask{0, S, rho[i], z[i]};
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  double* d = nullptr;
  const size_t per = ncoef(nmax);
  FMM_HIP_TRY(hipMalloc(&d, npts * per * sizeof(double)));
  int64_t nu = 0;
  int rc = (s->kind == 1)
               ? gpu_table_tasks(s->medium, comps, smap, s->d_lad, s->dm, s->tg, s->d_tab, s->nmax, tasks, nmax, d,
                                 &nu, st, used)
               : gpu_surrogate_tables(s->medium, comps, smap, s->d_lad, s->dm, tasks, nmax, s->net, d, &nu, st, used);
  if (rc == FMMLM_OK) {
    hipError_t e = hipMemcpy(out, d, npts * per * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      set_last_error(hipGetErrorString(e));
      rc = FMMLM_EDEVICE;
    }
  }
  hipFree(d);
  return rc;
}

}  // extern "C"
