// Kernel-side structures and host launchers shared by the kernels and the
// C-ABI layer of the IS shape-overlap engine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shape_device.hpp"
#include "shape_is.h"

namespace shape {

constexpr int kEstSums = 11;

// Molecule set as handed over through the C ABI.
struct MolsDev {
  int n_mols;
  int max_atoms;
  int64_t n_atoms;
  const int* off;
  const float* xyz;
  const float* alpha;
  const uint32_t* id;
};

// Prepared per-atom / per-molecule records (context scratch).
struct Prepared {
  Atom* atom;
  AtomSampling* samp;
  double* Z;
  uint32_t* id;
  int* bad;
  float4* centre;  // mean atom position (frame origin of the expanded form)
};

struct ScreenArgs {
  Prepared Q;
  const int* offQ;
  int max_q;
  Prepared L;
  const int* offL;
  int n_lib;
  int max_b;
  const float4* qs;
  const float* qf2;
  const int* pairs;
  int n_pairs;
  int mode;
  int64_t n_fixed;     // fixed mode: samples per side
  int round_side;      // samples per side per round (multiple of 64)
  int64_t cap_pair;    // adaptive cap, samples per pair
  double tau;
  uint2 key;
  const int* n_start;  // optional per-pair budgets (adaptive)
  int anti;            // antithetic sampling: terms are pair means
  const int* order;    // optional launch order: block b screens pair order[b]
  float* T;
  float* se_T;
  float* O_ab;
  float* O_aa;
  float* O_bb;
  int* n_used;
};

// Alignment: pairs (A[p], B[p]), n_starts poses each.
struct AlignArgs {
  Prepared A;
  const int* offA;
  int max_a;
  Prepared B;
  const int* offB;
  int max_b;
  int n_starts;
  int n_samples;
  uint2 key;
  const float* pose;  // [pairs][starts][7] (qw, qx, qy, qz, tx, ty, tz)
  const float* O_aa;  // [pairs]
  const float* O_bb;  // [pairs]
  float* T;           // [pairs][starts]
  float* grad;        // [pairs][starts][7] or nullptr
  // n_steps > 0: Adam ascent on T inside the kernel (pose updated in place,
  // T and grad then at the final pose); 0: one evaluation at the given pose.
  int n_steps;
  float lr;
  float* pose_out;    // the pose array again (written when n_steps > 0)
  const int* order;   // optional launch order: block b aligns pair order[b]
};

// Dense layer C = epilogue(A B) with strided operands (see shape_gemm).
struct GemmArgs {
  int M, N, K;
  const float* A;
  int64_t sam, sak;
  const float* B;
  int64_t sbk, sbn;
  float* C;
  int64_t scm;
  const float* bias;
  const float* gate;
  int64_t sgm;
  int flags;
  // split-K: when part is set, workgroup z covers k in [z k_chunk, (z+1) k_chunk)
  // and writes its raw partial tile to part[z][M][N]; a reduction adds the
  // partials in z order and applies the epilogue
  int k_chunk = 0;
  float* part = nullptr;
};

// Number of K splits launch_gemm will use for this product (1 = none) and
// the scratch it then needs (splits * M * N floats).
int gemm_splits(const GemmArgs& g);

// Features and first-order cross-overlaps read the caller's arrays directly;
// invalid molecules give NaN and raise *flag.  order (optional): a
// permutation of the molecules, taken four to a wave in its order.
hipError_t launch_features(const MolsDev& M, int* flag, float* out, float* mom,
                           hipStream_t st, const int* order = nullptr);
hipError_t launch_pair_features(const float* fq, const float* flib, const int* qidx,
                                const int* idx, int n, const float* fo_cross, const float* mean,
                                const float* inv_std, float* out, hipStream_t st);
hipError_t launch_fo_cross(const MolsDev& Q, const MolsDev& L, const int* pairs, int n_pairs,
                           int n_cu, int* flag, float* out, hipStream_t st);
hipError_t launch_gemm(const GemmArgs& g, hipStream_t st);
// several BF16 products with 64 x 64 tiles in one launch (plus one split-K
// reduction launch); part holds the sum of gemm_set_part_elems of the set
constexpr int kGemmSetMax = 8;
bool gemm_set_fits(const GemmArgs& g);
size_t gemm_set_part_elems(const GemmArgs& g);
int64_t gemm_set_blocks(const GemmArgs& g);
hipError_t launch_gemm_set(int n, const GemmArgs* gs, float* part, hipStream_t st);
size_t mlp_pack_bytes();
// fused training step of the surrogate (forward, MSE, backward, Adam)
struct MlpStep {
  const float *fq, *flib;
  const int *qidx, *idx;
  int n;
  const float* fo_cross;
  const float *mean, *inv_std, *target, *lw;
  float *params, *m, *v;
  int* step;
  void* packed;
  float lr, b1, b2, eps;
  float* grad;
  float* loss;
};
size_t mlp_pack_all_bytes();
hipError_t launch_mlp_pack_all(const float* params, void* packed, hipStream_t st);
int mlp_step_rows();
size_t mlp_step_scratch_bytes(int n);
hipError_t launch_mlp_step(const MlpStep& s, void* scratch, hipStream_t st);
// dense-grid quadrature
struct GridDims {
  double lo[3];
  double h;
  int n[3];
  int nmax;
};
hipError_t launch_grid_box(const float* xa, int na, const float* xb, int nb, double* box,
                           hipStream_t st);
hipError_t launch_grid(const float* xa, const float* aa, int na, const float* xb,
                       const float* ab, int nb, const GridDims& g, double* tables, double* part,
                       double* out, hipStream_t st);
// hybrid pipeline (first-order alignment)
hipError_t launch_fo_starts(const MolsDev& A, const MolsDev& B, const int* badA,
                            const int* badB, int n_random, uint2 key, float* pose,
                            hipStream_t st);
size_t fo_align_lds_bytes(int max_a, int max_b);
hipError_t launch_fo_align(const MolsDev& A, const MolsDev& B, const int* badA, const int* badB,
                           int n_starts, int n_steps, float lr, float* pose, float* T,
                           float* grad, hipStream_t st,
                           const int* order = nullptr);
// whether launch_fo_align runs one workgroup per pair (the row layout)
bool fo_align_pair_major(int max_a, int max_b, int n_starts);
hipError_t launch_best_pose(const float* T, const float* pose, int n_pairs, int n_starts,
                            float* best_pose, float* best_T, hipStream_t st);
hipError_t launch_apply_pose(const MolsDev& M, const float* pose, float* out, hipStream_t st);
hipError_t launch_group_max(const float* T, int64_t n_T, const int* goff, int n_groups,
                            float* best_T, int* best_idx, int* flag, hipStream_t st);
hipError_t launch_seed_budget(const float* raw, int64_t ld, const int* idx, int k, double y_mean,
                              double y_std, double tau, int round, int cap, int* n_start,
                              hipStream_t st);
hipError_t launch_mlp_infer(const float* fq, const float* flib, const int* qidx, const int* idx,
                            int n, const float* fo_cross, const float* mean,
                            const float* inv_std, const float* params, void* packed,
                            float* out, hipStream_t st, float* x_out = nullptr,
                            float* const* h_out = nullptr);
int colsum_chunks(int M);
constexpr int kColSetMax = 8;
hipError_t launch_colsum_set(int n, const int* M, const int* N, const float* const* A,
                             const int64_t* lda, float* const* out, hipStream_t st);
hipError_t launch_colsum(const float* A, int M, int N, int64_t lda, float* part, float* out,
                         hipStream_t st);
int mse_blocks(int B, int N);
hipError_t launch_mse(const float* y, const float* t, const float* w, int B, int N, float* grad,
                      double* partial, float* loss, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, int* step,
                       float lr, float b1, float b2, float eps, hipStream_t st);
int topk_blocks(int n);
hipError_t launch_topk(const float* s, int n, int k, uint32_t* sel, uint32_t* hist, int* cnt_gt,
                       int* cnt_eq, int* out, hipStream_t st);

size_t align_lds_bytes(int n_samples, int max_a, int max_b);
hipError_t launch_align(const AlignArgs& a, int n_pairs, hipStream_t st);
hipError_t launch_self_overlap(const Prepared& M, const int* off, int n_mols, int n_samples,
                               uint2 key, float* out, hipStream_t st);
hipError_t launch_adam_pose(float* pose, const float* dT, float* m, float* v, int64_t n_poses,
                            int* step, float lr, float b1, float b2, float eps, hipStream_t st);
hipError_t launch_best_start(const float* T, int n_pairs, int n_starts, int* best,
                             hipStream_t st);

hipError_t launch_alpha_from_radius(const float* R, int64_t n, double kappa, double lambda,
                                    float* alpha, hipStream_t st);
// which (optional, [n_which]): prepare only these molecules.
hipError_t launch_prepare(const MolsDev& in, const Prepared& out, int* flag, int* set_flag,
                          hipStream_t st, const int* which = nullptr, int n_which = 0);
hipError_t launch_flag_or(int* flag, const int* set_flag, hipStream_t st);
hipError_t launch_fill_int(int* p, int n, int v, hipStream_t st);
int est_blocks(int64_t n_units);
hipError_t launch_estimate(const Prepared& A, const Prepared& B, const int* offA,
                           const int* offB, int64_t n_a, int64_t n_b, uint2 key, int anti,
                           double* partials, int nblk, shape_result* out_dev, hipStream_t st);
hipError_t launch_query_cache(const Prepared& Q, const int* offQ, int64_t n, uint2 key, int anti,
                              float4* qs, float* qf2, hipStream_t st);
// sampling steps of one prepared molecule (thresholds, Philox words,
// components, points); n samples from counter k0
hipError_t launch_sample_points(const Prepared& P, const int* off, int mol, int max_atoms,
                               int64_t k0, int n, uint2 key, int anti, uint32_t* thr,
                               uint32_t* words, int* comp, float* r, hipStream_t st);
size_t screen_lds_bytes(int max_q, int max_b);
constexpr int kScreenVariants = 8;
extern const int kScreenVariantShape[kScreenVariants][2];  // {kSA, kSB}
hipError_t launch_screen(const ScreenArgs& a, int variant, hipStream_t st);
// Launch order of a grid with one workgroup per pair (blocks along x):
// largest estimated work first.  The work of pair p is
// wA N_A + wB N_B + w0 atoms' worth, times the rounds of its seeded budget
// when n_start is given; with per_xcd each XCD keeps the pairs xcd_chunk
// deals it and takes them largest first, else one order over all blocks.
struct OrderArgs {
  int n;                // pairs
  int per_xcd;
  const int* pairs;     // optional: pair -> molecule of set B (else p)
  const int* offA;      // optional set A: molecule p, or molecule 0 if a_single
  int nA_mols, max_a, a_single;
  const int* offB;
  int nB_mols, max_b;
  int quad_b;           // B's term is wB n_B^2 (else wB n_B)
  uint32_t wA, wB, w0;
  const int* n_start;   // optional per-pair sample budgets
  int64_t round_pair, cap;
};
// order: int [n] (a permutation of [0, n)); work: work_order_ints() ints,
// 16-byte aligned
int work_order_ints();
hipError_t launch_work_order(const OrderArgs& o, int* order, int* work, hipStream_t st);

// issue-rate microbenchmarks (measurement support): which = 0 FP32 FMA,
// 1 v_exp_f32, 2 v_mad_u64_u32, 3 LDS 16-byte reads, 4 FP32 FMA with SGPR
// operands; out holds one float per
// lane of the grid (peak_blocks(n_cu) x 256)
int peak_blocks(int n_cu);
hipError_t launch_peak(int which, int n_cu, int iters, float* out, hipStream_t st);
double peak_work_per_iter(int which);

}  // namespace shape
