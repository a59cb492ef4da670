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
#include <chrono>
#include <unordered_set>
#include <cmath>
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
  return md;
}

double coefA_host(int n, int m) {
  const double cn = std::sqrt((2.0 * n + 1.0) / (4.0 * M_PI));
  return ((n & 1) ? -1.0 : 1.0) * cn / std::sqrt(std::tgamma(n - m + 1.0) * std::tgamma(n + m + 1.0));
}

void free_plan(fmmlm_plan_s* P) {
  if (!P) return;
  for (auto e : P->prof_ev) (void)hipEventDestroy(e);
  for (auto& b : P->bufs) hipFree(b.ptr);
  delete P;
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
  // ---- M2L tiles: up to tile_cols target boxes of one level, tree and octant
  // class per tile (boxes of one class share their interaction offsets); one
  // step per operator (free space or reaction) present in the tile
  std::vector<int32_t> tptr(1, 0), ttgt, tlev, sop, skind, ssrc, us, tuptr;
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
    std::vector<int> slot(std::max<int64_t>(P->nops, 1), -1);
    std::vector<int> used;
    for (int l = 0; l <= P->maxlev; ++l) {
      std::vector<std::vector<int32_t>> bucket((size_t)nt * 8);
      for (int64_t b = P->lev_off[l]; b < P->lev_off[l + 1]; ++b)
        if (mptr[b + 1] > mptr[b]) {
          const HBox& bx = B.boxes[b];
          bucket[(size_t)bx.tree * 8 + ((bx.ix & 1) | ((bx.iy & 1) << 1) | ((bx.ih & 1) << 2))].push_back(
              (int32_t)b);
        }
      for (const auto& tg : bucket)
        for (size_t c0 = 0; c0 < tg.size(); c0 += TBc) {
          const size_t nc_ = std::min<size_t>(TBc, tg.size() - c0);
          tlev.push_back(l);
          for (size_t c = 0; c < (size_t)TBc; ++c) ttgt.push_back(c < nc_ ? tg[c0 + c] : -1);
          used.clear();
          std::vector<std::vector<int32_t>> cols;
          for (size_t c = 0; c < nc_; ++c) {
            const int32_t b = tg[c0 + c];
            for (int32_t e = mptr[b]; e < mptr[b + 1]; ++e) {
              const int op = (mop[e] >= 0) ? mop[e] : ~mop[e];
              if (slot[op] < 0) {
                slot[op] = (int)cols.size();
                cols.emplace_back(TBc, -1);
                used.push_back(op);
              }
              cols[slot[op]][c] = msrc[e];
            }
          }
          std::sort(used.begin(), used.end());
          for (int op : used) {
            sop.push_back(op);
            skind.push_back(op < nfo ? (int32_t)FMMLM_FREE : (int32_t)FMMLM_REACTION);
            ssrc.insert(ssrc.end(), cols[slot[op]].begin(), cols[slot[op]].end());
          }
          for (int op : used) slot[op] = -1;
          tptr.push_back((int32_t)sop.size());
        }
    }
    P->ntiles = (int64_t)tlev.size();
    P->nsteps = (int64_t)sop.size();
    P->tile_split = 0;
    while (P->tile_split < P->ntiles && tlev[P->tile_split] < P->opts.fp64_top_levels) ++P->tile_split;
    // work units of at most kStepsPerUnit steps
    constexpr int kStepsPerUnit = 16;
    tuptr.assign(1, 0);
    for (int64_t t = 0; t < P->ntiles; ++t) {
      for (int32_t a = tptr[t]; a < tptr[t + 1]; a += kStepsPerUnit) {
        us.push_back(a);
        us.push_back(std::min(a + kStepsPerUnit, tptr[t + 1]));
      }
      tuptr.push_back((int32_t)(us.size() / 2));
      if (t + 1 == P->tile_split) P->unit_split = (int64_t)(us.size() / 2);
    }
    P->nunits = (int64_t)(us.size() / 2);
    // operator tables must fit a budget (FP64 + FP32 copies)
    const double tbytes = (double)P->nops * P->nrk * 32.0 * P->mrt * (P->fp32 ? 12.0 : 8.0);
    if (tbytes > 32.0 * (1 << 30)) {
      set_last_error("M2L operator tables exceed 32 GiB");
      return FMMLM_ENOMEM;
    }
  }
  // ---- P2P CSR over leaves
  std::vector<int32_t> pptr(P->nleaves + 1, 0), psrc;
  std::vector<int32_t> rptr(P->nleaves + 1, 0), rsrc;
  std::vector<int64_t> rvoff;
  std::vector<int32_t> rp_t, rp_s, rp_c;
  int64_t voff = 0;
  for (int64_t li = 0; li < P->nleaves; ++li) {
    const int b = leaves[li];
    for (auto& pr : B.p2p_free[b]) {
      psrc.push_back(pr.first);
      psrc.push_back(pr.second);
    }
    pptr[li + 1] = (int32_t)(psrc.size() / 2);
    for (auto& r : B.p2p_reac[b]) {
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
  UP(p2p_ptr, pptr); UP(p2p_src, psrc); UP(rp_ptr, rptr); UP(rp_src, rsrc); UP(rp_voff, rvoff);
  UP(coefA, coefA); UP(sc_levels, scl);
  UP(tile_ptr, tptr); UP(tile_tgt, ttgt); UP(tile_level, tlev); UP(step_op, sop); UP(step_src, ssrc);
  UP(unit_s, us); UP(tile_unit_ptr, tuptr); UP(step_kind, skind);
  if ((rc = dev_alloc(P, &P->Wm2l, (size_t)std::max<int64_t>(P->nunits, 1) * P->tile_cols * 32 * P->mrt))) return rc;
#undef UP
  P->stats.lists_seconds = seconds_since(tphase);
  tphase = std::chrono::steady_clock::now();
  // ---- operators: free-space harmonics and reaction Sommerfeld tables
  if ((rc = dev_alloc(P, &P->G, (size_t)std::max<int64_t>(P->nops, 1) * P->ng * 2))) return rc;
  double* tables = nullptr;
  if (!B.tasks.empty()) {
    FMM_HIP_TRY(hipMalloc(&tables, B.tasks.size() * (size_t)P->ng * sizeof(double)));
    const auto ts = std::chrono::steady_clock::now();
    rc = gpu_sommerfeld_tables(P->medium, comps, B.tasks, 2 * p, tables, st);
    P->stats.table_seconds = seconds_since(ts);
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
  if (P->fp32) {
    const size_t nr = (size_t)(P->p + 1) * (P->p + 1);
    if ((rc = dev_alloc(P, &P->Tfree32, (size_t)std::max<int64_t>(P->nops, 1) * P->nrk * 32 * P->mrt))) return rc;
    if (std::min(P->opts.max_rhs, 64) == 1 && (rc = dev_alloc(P, &P->M32, (size_t)P->NB * nr))) return rc;
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
    rc = gpu_reaction_nearfield(P->medium, comps, dt, ds, dc, npairs, P->px, P->py, P->ph, P->rp_val, st);
    P->stats.nearfield_seconds = seconds_since(ts);
    hipFree(dt);
    hipFree(ds);
    hipFree(dc);
    if (rc) return rc;
  }
  // ---- workspace (G = min(max_rhs, 64) vectors per pass)
  P->gmax = std::min(P->opts.max_rhs, 64);
  const size_t G = (size_t)P->gmax;
  const size_t nrr = (size_t)(P->p + 1) * (P->p + 1);
  if ((rc = dev_alloc(P, &P->qt, P->NP * G))) return rc;
  if ((rc = dev_alloc(P, &P->phit, P->NP * G))) return rc;
  if ((rc = dev_alloc(P, &P->M, (size_t)P->NB * nrr * G))) return rc;
  if ((rc = dev_alloc(P, &P->Lx, (size_t)P->NB * nrr * G))) return rc;
  if (P->fp32 && G > 1 && (rc = dev_alloc(P, &P->M32, (size_t)P->NB * nrr * G))) return rc;
  if (G > 1) {
    if ((rc = dev_alloc(P, &P->qb64, P->NP * 64))) return rc;
    if (P->fp32 && (rc = dev_alloc(P, &P->qb32, P->NP * 64))) return rc;
    std::vector<int32_t> bb;
    for (int64_t b = 0; b < P->NB; ++b)
      if (mptr[b + 1] > mptr[b]) {
        if (B.boxes[b].level < P->opts.fp64_top_levels) P->bbox_split = (int64_t)bb.size() + 1;
        bb.push_back((int32_t)b);
      }
    P->nbbox = (int64_t)bb.size();
    if ((rc = dev_upload(P, &P->bbox, bb, st))) return rc;
  }
  FMM_HIP_TRY(hipStreamSynchronize(st));
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

int fmm_layered_plan(int32_t n_interfaces, const double* z_interfaces, const double* eps, int64_t n,
                     const double* x, const double* y, const double* z, const int32_t* layer_id, int32_t p,
                     const fmmlm_opts* opts, void* hip_stream, fmmlm_plan_t* out) {
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
  for (int i = 0; i < 3; ++i)
    if (o.reserved[i] != 0) return FMMLM_EINVAL;
  if (o.fp64_top_levels < 0 || o.fp64_top_levels > kMaxLevel + 1) return FMMLM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  std::vector<double> dv, ev, X, Y, Z;
  std::vector<int32_t> LAY;
  int rc;
  if ((rc = fetch(z_interfaces, n_interfaces, dv))) return rc;
  if ((rc = fetch(eps, n_interfaces + 1, ev))) return rc;
  if ((rc = validate_medium(n_interfaces, dv, ev))) return rc;
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

int fmm_layered_eval(fmmlm_plan_t plan, int32_t nrhs, const double* q, int64_t ldq, double* phi, int64_t ldphi,
                     uint32_t parts, void* hip_stream) {
  if (!plan || !q || !phi) return FMMLM_EINVAL;
  if (nrhs < 1 || nrhs > plan->opts.max_rhs) return FMMLM_EINVAL;
  if (ldq < plan->N || ldphi < plan->N) return FMMLM_EINVAL;
  if (parts == 0 || (parts & ~(FMMLM_FREE | FMMLM_REACTION))) return FMMLM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (nrhs == 1) {
    hipEvent_t* ev = nullptr;
    if (plan->prof_used < plan->prof_cap) ev = &plan->prof_ev[(size_t)plan->prof_used++ * (FMMLM_NSTAGES + 1)];
    return gpu_eval_one(plan, q, phi, parts, st, ev);
  }
  for (int r0 = 0; r0 < nrhs; r0 += plan->gmax) {
    const int g = std::min(plan->gmax, nrhs - r0);
    hipEvent_t* ev = nullptr;
    if (plan->prof_used < plan->prof_cap) ev = &plan->prof_ev[(size_t)plan->prof_used++ * (FMMLM_NSTAGES + 1)];
    int rc = gpu_eval_batch(plan, g, q + (int64_t)r0 * ldq, ldq, phi + (int64_t)r0 * ldphi, ldphi, parts, st, ev);
    if (rc) return rc;
  }
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
    default: break;
  }
  msg = base;
  if (code == FMMLM_EDEVICE || code == FMMLM_ENOMEM) {
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

}  // extern "C"
