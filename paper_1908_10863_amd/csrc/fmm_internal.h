// Internal declarations of the layered-media FMM library (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <string>
#include <array>
#include <vector>

#include "../../include/fmmlm.h"

namespace fmmlm {

constexpr int kMaxL = FMMLM_MAX_INTERFACES;
constexpr int kPMax = FMMLM_PMAX;
constexpr int kMaxLevel = 20;  // 21-bit quantisation per axis
// sparse top-level M2L: threads of a block, rounds of entries per work item
constexpr int kSpThreads = 512;
constexpr int kSpItemRounds = 1;
// batched FP32 form, FP64 top levels: entries per work item
constexpr int kBatchTopItem = 24;
// reaction P2P: target rows per work unit (one wave, 8 lanes a row)
constexpr int kRPUnitRows = 8;
// free P2P (single vector): targets of one work unit, 16 lane slots x targets
// a lane (8 in FP32, 4 in FP64)
constexpr int kPLUnitTargetsF32 = 128;
constexpr int kPLUnitTargetsF64 = 64;
// operator-major M2L: operators grouped into one chunk's steps, and the
// fewest targets common to a group's operators that make grouped chunks
constexpr int kM2LGroupOps = 4;
constexpr int kM2LGroupMinTargets = 64;

// unit ranges of the FP32 M2L launch per XCD (the 8 XCDs take blocks in turn):
// XCD x runs units [off[x], off[x + 1]) of the launch, ranges of about equal
// steps
struct XcdSplit {
  int32_t off[9];
};

// ---- small complex type (device and host) ------------------------------------
struct cplx {
  double re, im;
};
__host__ __device__ inline cplx cmk(double r, double i) { return cplx{r, i}; }
__host__ __device__ inline cplx operator+(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cplx operator-(cplx a, cplx b) { return cplx{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cplx operator*(cplx a, cplx b) {
  return cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline cplx operator*(double s, cplx a) { return cplx{s * a.re, s * a.im}; }
__host__ __device__ inline cplx cconj(cplx a) { return cplx{a.re, -a.im}; }
__host__ __device__ inline cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, den = b.re + b.im * r;
    return cplx{(a.re + a.im * r) / den, (a.im - a.re * r) / den};
  }
  const double r = b.re / b.im, den = b.re * r + b.im;
  return cplx{(a.re * r + a.im) / den, (a.im * r - a.re) / den};
}
__device__ inline cplx cexp_dev(cplx a) {
  const double e = exp(a.re);
  double s, c;
  sincos(a.im, &s, &c);
  return cplx{e * c, e * s};
}

// ---- layered medium (passed by value to kernels) ------------------------------
// General interface conditions a_{i} u_i = a_{i+1} u_{i+1}, b_i u_i' =
// b_{i+1} u_{i+1}' are held as eps = b / a and acoef = a: with v = a u they are
// the classic conditions for v with permittivities b / a and a source of
// strength a in the source layer, so every density is a_ls / a_lt times the
// classic one for eps = b / a (classic: acoef = 1).
struct Medium {
  int L;                      // interfaces; 0 means sigma == 1 (test medium)
  double d[kMaxL];            // interface heights, decreasing
  double eps[kMaxL + 1];      // permittivities (b / a), top to bottom
  double acoef[kMaxL + 1];    // the a coefficients (1 for the classic conditions)
};

// coefficient index of (n, m), 0 <= m <= n
__host__ __device__ inline int cidx(int n, int m) { return n * (n + 1) / 2 + m; }
__host__ __device__ inline int ncoef(int p) { return (p + 1) * (p + 2) / 2; }

// ---- host-side plan ----------------------------------------------------------
struct TreeInfo {
  int layer = 0, side = 0;       // side 1: h = z - d_l ; side 2: h = d_{l-1} - z
  int64_t n = 0, pt_off = 0;     // points in global tree order [pt_off, pt_off + n)
  std::vector<uint64_t> keys;    // sorted Morton keys (host copy, introspection)
  std::vector<int64_t> perm;     // user index of each tree point (host copy)
};

struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace fmmlm

namespace fmmlm {
// arguments of the evaluation a plan's captured graph replays
struct GraphKey {
  int32_t nrhs = 0;
  const double* q = nullptr;
  int64_t ldq = 0;
  double* phi = nullptr;
  int64_t ldphi = 0;
  uint32_t parts = 0;
  hipStream_t st = nullptr;
  bool operator==(const GraphKey& o) const {
    return nrhs == o.nrhs && q == o.q && ldq == o.ldq && phi == o.phi && ldphi == o.ldphi && parts == o.parts &&
           st == o.st;
  }
};
}  // namespace fmmlm

struct fmmlm_plan_s {
  int L = 0;
  std::vector<double> d, eps;
  fmmlm::Medium medium;
  int64_t N = 0;
  int p = 0, nc = 0, ng = 0;
  fmmlm_opts opts;
  double x0 = 0, y0 = 0, W = 0, scale = 0;
  std::vector<fmmlm::TreeInfo> trees;
  int64_t NP = 0;           // total tree points
  int64_t NB = 0;           // total boxes
  int maxlev = 0;
  std::vector<int64_t> lev_off;  // global box index where level l starts, size maxlev + 2
  int64_t nleaves = 0;
  fmmlm_stats stats;

  // device buffers (owned)
  std::vector<fmmlm::DevBuf> bufs;
  int64_t device_bytes = 0;

  // points, tree order (global)
  double *px = nullptr, *py = nullptr, *ph = nullptr;
  int32_t* puser = nullptr;        // user index per tree point
  int32_t* user_pos = nullptr;     // [N][2] tree positions of each user point (-1 if none)
  // boxes (global, level-major)
  double *bcx = nullptr, *bcy = nullptr, *bch = nullptr;
  int32_t *blevel = nullptr, *bstart = nullptr, *bcount = nullptr, *bparent = nullptr;
  int32_t *bchild0 = nullptr, *bnchild = nullptr;
  int32_t* leaves = nullptr;       // leaf box ids
  int32_t* pleaf = nullptr;        // leaf list index of every tree point
  int64_t max_leaf = 0;            // largest leaf population
  std::vector<std::pair<int64_t, int64_t>> free_ranges;  // (first point, count) of free-space trees
  // M2L CSR over target boxes
  int32_t *m2l_ptr = nullptr;      // [NB + 1] ; free entries first, then reaction
  int32_t *m2l_nfree = nullptr;    // [NB] number of free entries per target box
  int32_t *m2l_src = nullptr, *m2l_op = nullptr;  // op < 0 encodes mirrored source: ~op
  double* G = nullptr;             // operators [nops][ng] complex (re, im interleaved)
  // M2L as GEMMs over operator-major chunks (a chunk is a tile of its own)
  double* Tfree = nullptr;         // [nops][nrk][32 mrt] real-form operators (free space, then reaction)
  int nrk = 0, mrt = 0;            // padded inner dimension, rows per thread / 32
  int tile_cols = 64;              // target boxes per tile (128 when mrt <= 4)
  int64_t tile_grp[5] = {0};       // target-tile groups (none: all zero, the chunks follow)
  int m2l_variant = 0;             // FP32 M2L tile shape picked by the autotuner
  fmmlm::XcdSplit m2l_xcd{};        // FP32 M2L: the chunk units' ranges per XCD
  int32_t m2l_xcd_len = 0;          //   ... and the longest range (blocks per XCD)
  int batch_variant = 0;           // batched FP32 M2L shape / persistence picked by the autotuner
  // M2M / L2L as GEMMs: 16 real-form operators (8 child octants up, 8 down)
  // and their own tiles; per level (first tile, first unit, end tile, end unit)
  double* Txl = nullptr;           // [16][nrk][32 mrt]
  std::vector<std::array<int64_t, 4>> xl_m2m, xl_l2l;
  std::vector<char> xl_need_m2m, xl_need_l2l;  // per level: the translation into it is needed
  int64_t xl_units = 0;
  int32_t *xl_step_op = nullptr, *xl_step_src = nullptr;
  int32_t *xl_unit_s = nullptr, *xl_unit_mask = nullptr, *xl_tile_unit_ptr = nullptr, *xl_tile_tgt = nullptr;
  int xl_tile_cols = 32;           // target boxes per translation tile
  int32_t* sp_boxes = nullptr;     // target boxes of the sparse top levels (no tiles there)
  // their work items (sparse box, first entry, end entry), per box a run of
  // items (sp_item_ptr), partial sums per item [n_sp_items][nc] complex
  int32_t *sp_items = nullptr, *sp_item_ptr = nullptr;
  int64_t n_sp_items = 0;
  int sp_ne = 1;                   // entries per round of an item's block ...
  int sp_threads = 64;             //   ... and its threads (a multiple of 64)
  double* Psp = nullptr;
  // FP32 form: operator-major chunks; per target box its slots (unit * tile_cols + column)
  int32_t *slot_boxes = nullptr, *slot_ptr = nullptr, *slots = nullptr;
  int64_t n_slot_boxes = 0;
  int64_t n_sp_boxes = 0;
  // work units: a tile's steps split into chunks (more blocks in flight)
  int64_t nunits = 0, unit_split = 0;
  int32_t *unit_s = nullptr;       // [2 * nunits] step range of each unit
  int32_t *unit_mask = nullptr;    // [nunits] column groups of 8 that the unit's partial holds
  int32_t *tile_unit_ptr = nullptr;// [ntiles + 1]
  double* Wm2l = nullptr;          // [nunits][tile_cols][32 mrt] partial products (FP64 form)
  float* W32m = nullptr;           // the same in FP32 (FP32 form)
  // FP32 form
  bool fp32 = false;
  float* Tfree32 = nullptr;        // FP32 copy of Tfree
  float* M32 = nullptr;            // FP32 copy of the multipole expansions (GEMM operand)
  float *pxh = nullptr, *pxl = nullptr, *pyh = nullptr, *pyl = nullptr, *phh = nullptr, *phl = nullptr;
  float* qt32 = nullptr;
  // batched form (opts.max_rhs > 1): expansions, charges and potentials of up
  // to G = min(max_rhs, 64) vectors; M2L one block per target box
  int gmax = 1;
  int batch_min = 2;               // batched passes narrower than this run vector by vector
  int64_t nbbox = 0, bbox_split = 0;
  int32_t* bbox = nullptr;         // target boxes with M2L entries, level order
  // batched M2M / L2L through the batched FP64 GEMM: per box CSR of its
  // translation entries (M2M: children, operator = octant; L2L: the parent,
  // operator 8 + octant) and the target boxes of each level
  int32_t *bu_ptr = nullptr, *bu_src = nullptr, *bu_op = nullptr, *bu_boxes = nullptr;
  int32_t *bd_ptr = nullptr, *bd_src = nullptr, *bd_op = nullptr, *bd_boxes = nullptr;
  std::vector<int64_t> bu_lev, bd_lev;  // level l's targets: [lev[l], lev[l + 1])
  double* qb64 = nullptr;          // [NP][64] vector-minor charges (FP64); after the near field,
                                   // the point-major potentials of the combine
  double* qu = nullptr;            // [N][64] point-major charges in user order (batched gather)
  float* qb32 = nullptr;           // [NP][64] (FP32 form)
  int64_t ntiles = 0, nsteps = 0;
  int32_t *tile_ptr = nullptr, *tile_tgt = nullptr, *tile_level = nullptr;
  int32_t *step_op = nullptr, *step_src = nullptr, *step_kind = nullptr;
  int32_t *step_mask = nullptr;    // per step: bit g set if columns [8 g, 8 g + 8) hold a source
  int64_t nops = 0, n_free_ops = 0;
  // P2P free, CSR over leaves
  int32_t *p2p_ptr = nullptr;      // [nleaves + 1]
  int32_t *p2p_src = nullptr;      // [2 * entries] (start, count)
  int32_t *pl_leaves = nullptr;    // leaf list indices with free-space P2P entries (batched form)
  int64_t n_pl_leaves = 0;
  // single-vector free P2P, mutual form: a unit is up to kPLUnitTargets(form)
  // targets of one leaf against the leaf itself (one way) and the ranges after
  // it in tree order (both ways).  Target-side sums go to mu_a (per point);
  // source-side sums to mu_b, where leaf c holds cb_n[c] rows of its count of
  // values from cb_base[c] (one row per unit that covers it, in unit order),
  // at the index mu_bidx gives for each position of a unit's ranges after the
  // first; a combine pass adds a point's values in that order
  int64_t n_mu_units = 0;
  int32_t *mu_order = nullptr;     // [n_mu_units] launch order (most pairs first)
  int32_t *mu_leaf = nullptr, *mu_tb = nullptr;  // [n_mu_units] leaf list index, first target
  int32_t *mu_rptr = nullptr;      // [n_mu_units + 1] into mu_rng; a unit's first range is its own leaf
  int32_t *mu_rng = nullptr;       // [2 * ranges] (start, count)
  int64_t *mu_boff = nullptr;      // [n_mu_units] the unit's first position in mu_bidx
  int32_t *mu_bidx = nullptr;      // [positions] index into mu_b
  int64_t *cb_base = nullptr;      // [nleaves] first row of the leaf in mu_b
  int32_t *cb_n = nullptr;         // [nleaves] rows of the leaf (-1: no free P2P)
  double *mu_a = nullptr;          // [NP]
  void *mu_b = nullptr;            // float (FP32 form) or double
  // P2P reaction, CSR over leaves
  int32_t *rp_ptr = nullptr;       // [nleaves + 1]
  int32_t *rp_src = nullptr;       // [2 * entries] (start, count)
  int64_t *rp_voff = nullptr;      // [entries] value offset
  double *rp_val = nullptr;        // kernel values, row-major per entry (targets x sources)
  float* rp_val32 = nullptr;        // FP32 form: the same rounded to FP32 (single-vector reaction P2P)
  int32_t *rp_row = nullptr;       // [entries] first partial-sum slot of the entry's target rows
  int32_t *rp_units = nullptr;     // [3 * n_rp_units] (entry, first row, target count)
  int64_t n_rp_units = 0;
  double *Prp = nullptr;           // per (entry, target row) partial sums
  // batched FP32 form, FP64 top levels: work items (box-list index, first and
  // end entry), per box a run of items, partials [item][64][(p+1)^2]
  int32_t *btop_items = nullptr, *btop_iptr = nullptr;
  int64_t n_btop_items = 0;
  double* Pbtop = nullptr;
  int32_t *rp_units16 = nullptr;   // batched FP32 form: [3 * n_rp_units16] units of 16 rows
  int64_t n_rp_units16 = 0;
  float *Prb = nullptr;            // ... and their partial sums [entry row][64 vectors]
  // constants
  double *coefA = nullptr;         // A_n^m for n <= 2p, m <= n : [cidx]
  double *coefR = nullptr;         // solid-harmonic recurrence coefficients for n <= p (P2M, L2P)
  double *coefC2inv = nullptr;     // 1 / c_n^2, n <= p
  // workspace
  double *qt = nullptr, *phit = nullptr;
  double *M = nullptr, *Lx = nullptr;  // [NB][(p+1)^2] real layout
  double *sc_levels = nullptr;     // 1/S_l per level
  // single-vector evaluations: the near field (into phin) and the sparse top
  // levels run on their own streams, joined to the caller's stream by events
  double* phin = nullptr;          // near-field potentials, tree order [NP]
  hipStream_t s_near = nullptr, s_top = nullptr;
  hipEvent_t ev_q = nullptr, ev_m = nullptr, ev_near = nullptr, ev_top = nullptr;
  hipEvent_t ev_l = nullptr;       // main M2L launched (the rest of the near field may start)
  int64_t pl_split = 0;            // free P2P units launched at the fork; the rest after the main M2L
  size_t pl_pad = 28672;           // LDS a free P2P block reserves beside the far field (tuned)
  // graph mode: the captured evaluation and its arguments
  hipGraphExec_t gexec = nullptr;
  fmmlm::GraphKey gkey;
  // live stage timing
  std::vector<hipEvent_t> prof_ev;  // [max_evals][FMMLM_NSTAGES + 1]
  int prof_cap = 0, prof_used = 0;
  // overlap detection (FMMLM_EBUSY): set while a call enqueues work on the plan;
  // the last evaluation's end, recorded on its stream
  std::atomic<int> busy{0};
  hipEvent_t ev_done = nullptr;
  hipStream_t done_stream = nullptr;
  bool done_recorded = false;
};

namespace fmmlm {

// ---- device entry points implemented in the .hip files ------------------------
struct PlanBuildInput;

// tree.hip
int gpu_sort_tree(const double* dx, const double* dy, const double* dz, int64_t n, int side,
                  double dref, double x0, double y0, double scale, uint64_t* keys_out,
                  int64_t* perm_out, hipStream_t st, std::string* err);

// sommerfeld.hip
struct SommTask {
  int comp;           // reaction component index into the component table
  double S;           // box size at the level
  double rho, z;      // horizontal and vertical centre distance
};
struct CompInfo {
  int lt, ls, a, b;
  double zinf;        // decay length of the density (shortest ray path)
  double sinf;        // its amplitude: sigma(k) e^{k zinf} -> sinf as k -> infinity
};
int gpu_sommerfeld_tables(const Medium& md, const std::vector<CompInfo>& comps,
                          const std::vector<SommTask>& tasks, int nmax, double* d_out,
                          hipStream_t st);
int gpu_sommerfeld_noalloc(const Medium& md, const CompInfo& c, double S, int64_t npts, const double* rho,
                           const double* z, int nmax, double* out, hipStream_t st);
int gpu_reaction_nearfield(const Medium& md, const std::vector<CompInfo>& comps,
                           const int32_t* d_tpt, const int32_t* d_spt, const int32_t* d_comp,
                           int64_t npairs, const double* px, const double* py, const double* ph,
                           double* d_val, hipStream_t st);
int gpu_density(const Medium& md, const CompInfo& c, int64_t nk, const double* kre,
                const double* kim, double* ore, double* oim, hipStream_t st);
double zeta_inf(const Medium& md, int lt, int ls, int a, int b);
double sigma_inf(const Medium& md, int lt, int ls, int a, int b);
inline CompInfo make_comp(const Medium& md, int lt, int ls, int a, int b) {
  return CompInfo{lt, ls, a, b, zeta_inf(md, lt, ls, a, b), sigma_inf(md, lt, ls, a, b)};
}

// learned form: image ladder + network, and the trained domain
struct SurrogateDomain {
  double rho_max, zeta_max;  // trained (rho, zeta) box; outside it the quadrature is used
  double dmin;               // thinnest finite layer (the remainder's decay length offset)
  double delta;              // ladder spacing 2 dmin: rung j sits at zeta + zinf + j delta
  double yscale;             // network output unit (rms of the training targets)
};
constexpr int kMlpH = 128;   // hidden width
constexpr int kLadder = 8;   // closed-form rungs sum_j c_j e^{-k j delta} of the density's remainder
constexpr double kSurDecay = 0.7;  // network output j carries the weight kSurDecay^{n_j}
constexpr int kMlpF = 4;     // continuous input features
// table form: Chebyshev points per panel and direction, panel grid over the domain
constexpr int kTabK = 12;
struct TableGrid {
  int npr = 0, npz = 0;      // panels in rho and in zeta
  double hr = 0.0, hz = 0.0; // panel sizes: rho_max / npr, zeta_max / npz
};
struct MlpNet {
  int ncomp = 0, nout = 0;   // components (one-hot input), outputs
  float* params = nullptr;   // device, flat: E A b1 W2 b2 W3 b3 W4 b4 (W[k][j]: input k -> output j)
  int64_t off[9] = {0};
  int64_t nparams = 0;
};
void mlp_layout(MlpNet& net);
int gpu_mlp_forward(const MlpNet& net, const int32_t* comp, const float* feat, int64_t n, float* out,
                    int ldo, int ocols, float* h1, float* h2, float* h3, hipStream_t st);
int gpu_mlp_init(const MlpNet& net, uint64_t seed, hipStream_t st);
int gpu_mlp_train(const MlpNet& net, const int32_t* comp, const float* feat, const float* y, int64_t n,
                  int steps, int B, double lr, uint64_t seed, double* loss_first, double* loss_last,
                  hipStream_t st);
int gpu_mlp_grad(const MlpNet& net, const int32_t* comp, const float* feat, const float* y, int64_t n,
                 float* grad, double* loss, hipStream_t st);
int gpu_mlp_adam_steps(const MlpNet& net, int nsteps, const float* grads, const double* lr, float* trace,
                       hipStream_t st);
// d_lad: ladder coefficients [surrogate component][kLadder] (device)
int gpu_surrogate_samples(const Medium& md, const std::vector<CompInfo>& comps, const double* d_lad,
                          const SurrogateDomain& dm, int nmax, uint64_t seed, int64_t n, int32_t* d_comp,
                          float* d_feat, float* d_y, hipStream_t st, double* d_rz = nullptr);
int gpu_surrogate_tables(const Medium& md, const std::vector<CompInfo>& comps,
                         const std::vector<int32_t>& smap, const double* d_lad, const SurrogateDomain& dm,
                         const std::vector<SommTask>& tasks, int nmax, const MlpNet& net, double* d_out,
                         int64_t* n_used, hipStream_t st, int32_t* h_used);
int gpu_surrogate_nearfield(const Medium& md, const std::vector<CompInfo>& comps,
                            const std::vector<int32_t>& smap, const double* d_lad, const SurrogateDomain& dm,
                            const int32_t* d_tpt, const int32_t* d_spt, const int32_t* d_comp,
                            int64_t npairs, const double* px, const double* py, const double* ph,
                            const MlpNet& net, double* d_val, int64_t* n_fallback, hipStream_t st);

int gpu_table_fill(const Medium& md, const std::vector<CompInfo>& comps, const double* d_lad,
                   const SurrogateDomain& dm, const TableGrid& g, int nmax, double* d_tab, hipStream_t st);
int gpu_table_tasks(const Medium& md, const std::vector<CompInfo>& comps, const std::vector<int32_t>& smap,
                    const double* d_lad, const SurrogateDomain& dm, const TableGrid& g, const double* d_tab,
                    int ynmax, const std::vector<SommTask>& tasks, int nmax, double* d_out, int64_t* n_used,
                    hipStream_t st, int32_t* h_used);
int gpu_table_nearfield(const Medium& md, const std::vector<CompInfo>& comps, const std::vector<int32_t>& smap,
                        const double* d_lad, const SurrogateDomain& dm, const TableGrid& g, const double* d_tab,
                        int nout, const int32_t* d_tpt, const int32_t* d_spt, const int32_t* d_comp, int64_t npairs,
                        const double* px, const double* py, const double* ph, double* d_val, int64_t* n_fallback,
                        hipStream_t st);
int gpu_interp2d(const TableGrid& g, int nout, const double* d_nodes, int64_t n, const double* d_rho,
                 const double* d_zeta, double* d_out, hipStream_t st);

// fmm.hip
int gpu_build_ops(fmmlm_plan_s* P, const std::vector<int>& free_off,
                  const std::vector<int>& reac_task, const std::vector<double>& reac_phi,
                  const std::vector<double>& reac_S, const double* d_tables, hipStream_t st);
int gpu_build_real_ops(fmmlm_plan_s* P, hipStream_t st);
int gpu_build_xlate_ops(fmmlm_plan_s* P, hipStream_t st);
int gpu_tune_m2l(fmmlm_plan_s* P, hipStream_t st);
int gpu_tune_eval(fmmlm_plan_s* P, hipStream_t st);
constexpr int kM2LVariants = 6;  // FP32 M2L tile shapes the autotuner tries
constexpr int kBatchShapes = 5;  // batched FP32 M2L tile shapes (each also persistent)
int gpu_tune_batch(fmmlm_plan_s* P, hipStream_t st);
// b[i] = (float)a[i], i < n (the FP32 form's copy of the reaction near-field values)
int gpu_round_f32(const double* a, int64_t n, float* b, hipStream_t st);
int gpu_build_fp32(fmmlm_plan_s* P, hipStream_t st);
int gpu_eval_batch(fmmlm_plan_s* P, int g, const double* q, int64_t ldq, double* phi, int64_t ldphi,
                   uint32_t parts, hipStream_t st, hipEvent_t* ev);
int gpu_eval_one(fmmlm_plan_s* P, const double* q, double* phi, uint32_t parts, hipStream_t st,
                 hipEvent_t* ev);

void set_last_error(const std::string& s);

// Takes the plan for one call (eval, solve): FMMLM_EBUSY when another call is
// enqueuing work on it, or when its last evaluation, enqueued on a stream
// other than st, has not finished.  plan_release gives it back and, with
// record, marks the end of the work just enqueued on st.
int plan_acquire(fmmlm_plan_s* P, hipStream_t st);
void plan_release(fmmlm_plan_s* P, hipStream_t st, bool record);
int eval_held(fmmlm_plan_s* P, int32_t nrhs, const double* q, int64_t ldq, double* phi, int64_t ldphi,
              uint32_t parts, hipStream_t st);

// sides (layer, side) of a medium in the surrogate's numbering
inline int side_index(int L, int layer, int side) {
  // layer 0: side 1 only; layers 1..L-1: sides 1, 2; layer L: side 2 only
  if (layer == 0) return 0;
  if (layer == L) return 2 * L - 1;
  return 1 + 2 * (layer - 1) + (side - 1);
}

}  // namespace fmmlm

struct fmmlm_surrogate_s {
  int L = 0;
  std::vector<double> d, eps;
  fmmlm::Medium medium;
  int p = 0, nmax = 0;                 // outputs 2 nmax + 1, nmax = 2p
  fmmlm::SurrogateDomain dm;
  std::vector<fmmlm::CompInfo> comps;  // (2L)^2, index t * 2L + s
  fmmlm::MlpNet net;
  std::vector<double> lad;             // ladder coefficients [component][kLadder]
  double* d_lad = nullptr;             // device copy
  double ladder_fit = 0.0;             // largest weighted residual of the ladder fits
  int device = 0;
  // table form (kind 1): the remainder tabulated instead of learned
  int kind = 0;                        // 0 network, 1 tables
  fmmlm::TableGrid tg;
  double* d_tab = nullptr;             // [component][panel][output][kTabK^2]
  double fill_seconds = 0.0;           // filling the tables by the quadrature
};

#define FMM_HIP_TRY(expr)                                                      \
  do {                                                                         \
    hipError_t _e = (expr);                                                    \
    if (_e != hipSuccess) {                                                    \
      fmmlm::set_last_error(std::string(#expr) + ": " + hipGetErrorString(_e)); \
      return FMMLM_EDEVICE;                                                    \
    }                                                                          \
  } while (0)
