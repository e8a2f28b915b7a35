// Kernel launchers of the IPC time step.  All launches go on the given stream.
#pragma once
#include "solver.h"

namespace tc {

// Scene-aligned block table: block k covers elements [b0[k], b1[k]) of scene sc[k].
struct BlockTable {
  int nblk = 0;
  const int* sc = nullptr;
  const int* b0 = nullptr;
  const int* b1 = nullptr;
  const int* sblk = nullptr;  // [S+1] first block of each scene (device)
};

// Hash-table entry: a target primitive inserted for one cell, with its box.
struct BpEntry {
  int t, cx, cy, cz;
  double lo[3], hi[3];
  // target attributes the query tests need, copied at fill time so a test costs one load:
  int v[3];    // contact vertices (v[2] = -1 for an edge)
  int scene;
  int body;    // the affine body all its vertices belong to, else -1
  int fixed;   // 1 when all its vertices are permanently fixed
  int pad[2];
};

// Broad-phase working set.
struct BroadPhase {
  int ntarget = 0;          // tris then edges
  double* tbox = nullptr;   // [ntarget][6]
  int* tcell = nullptr;     // [ntarget][6]
  int* tncell = nullptr;    // [ntarget]
  int* toff = nullptr;      // [ntarget]
  int table_mask = 0;
  int* bcount = nullptr;    // [table]
  int* bstart = nullptr;    // [table]
  int* bfill = nullptr;     // [table]
  BpEntry* entries = nullptr;
  int* qcount = nullptr;    // [Nq]
  int* qoff = nullptr;      // [Nq]
  int* overflow = nullptr;  // [S] set when a box of the scene spans too many cells
};

void launch_predict(const View& V, hipStream_t s);
void launch_set_moving(double* x, int n, const int* nodes, const double* tgt, hipStream_t s);
void launch_touching(const View& V, int n, const int* cand_q, const int* cand_t, int* bad, hipStream_t s);
void launch_diff3(int n3, const double* a, const double* b, double* out, hipStream_t s);
void launch_tets_positive(const View& V, const double* x, int* bad, hipStream_t s);
void launch_cmap(const View& V, const double* src, double* out, hipStream_t s);
void launch_cpos(const View& V, hipStream_t s);
void launch_cdisp(const View& V, const double* p, hipStream_t s);
void launch_cend(const View& V, double* cend, hipStream_t s);
void launch_snap_disp(const View& V, const int* cand, hipStream_t s);
void launch_body_resid(const View& V, unsigned long long* res, hipStream_t s);

// broad phase
void launch_bp_targets(const View& V, const double* P0, const double* P1, BroadPhase& bp,
                       int all_scenes, hipStream_t s);
void launch_bp_count(const View& V, BroadPhase& bp, hipStream_t s);
void launch_bp_fill(const View& V, BroadPhase& bp, hipStream_t s);
void launch_bp_query(const View& V, const double* P0, const double* P1, BroadPhase& bp, int all,
                     int emit, int* cand_q, int* cand_t, int* tmp_t, hipStream_t s);

// narrow phase: flag candidates with d < dhat at cpos
void launch_narrow(const View& V, int n, const int* cand_q, const int* cand_t, int* flag,
                   hipStream_t s);
void launch_compact_pairs(const View& V, int n, const int* cand_q, const int* cand_t,
                          const int* flag, const int* pos, int* pkind, int* pv, double* pmeps,
                          int* pscene, hipStream_t s);

// element derivatives
void launch_contact_records(const View& V, int n, const int* cand_q, const int* cand_t,
                            const int* flag, const int* pos, int* out, hipStream_t s);
void launch_gather3(int n, const int* idx, const double* src, double* out, hipStream_t s);
void launch_body_public(int nb, const double* y, const double* com0, double* out, hipStream_t s);
void launch_count_scene(int n, const int* pscene, int* cnt, hipStream_t s);
void launch_barrier_hess(const View& V, int np, const int* pkind, const int* pv,
                         const double* pmeps, double* pg, double* ph, hipStream_t s);
void launch_body_hess(const View& V, hipStream_t s);

// assembly
// Static block rows of the Newton system (elasticity and lumped mass) and the gradient of
// every node (inertia and elasticity; zero for body and padding nodes) of the iterating scenes.
void launch_fem_rows(const View& V, double* g, int mixed, hipStream_t s);
void launch_contrib_count(const View& V, int np, const int* pv, int* hcnt, int* gcnt,
                          hipStream_t s);
void launch_contrib_emit(const View& V, int np, const int* pv, const int* hoff, const int* goff,
                         uint64_t* hkey, int* hidx, int* hsrc, double* hcoef, uint64_t* gkey,
                         int* gidx, int* gsrc, double* gcoef, hipStream_t s);
void launch_seg_flags(int n, const uint64_t* keys, int* flags, hipStream_t s);
void launch_seg_start(int n, const int* flags, const int* segid, int* segstart, hipStream_t s);
void launch_reduce_blocks(const View& V, int nmax, const int* nseg, const uint64_t* keys, const int* idx,
                          const int* segstart, const int* src, const double* coef,
                          const double* ph, int* drow, int* dcol, void* dval, int* rowcnt,
                          int mixed, hipStream_t s);
void launch_reduce_grad(const View& V, int nmax, const int* nseg, const uint64_t* keys, const int* idx,
                        const int* segstart, const int* src, const double* coef,
                        const double* pg, double* g, hipStream_t s);
void launch_precond(const View& V, const int* drowptr, const int* dcol, const void* dval,
                    void* pinv, int* bad, int mixed, hipStream_t s);

// PCG over the node-block table TN (vector updates) and the row table TS (sparse product);
// partial sums per block.  T is the arithmetic of the linear solve (double, or float in the
// mixed-precision mode and in the passes of the refined FP64 mode); the right-hand side -g and
// the solution dx stay double.
template <class T>
struct PcgBufsT {
  const double* g;  // the system is H dx = -g
  int keep_gg;      // 1: keep P_gg, the stopping reference, from the previous solve (a
                    // refinement pass is measured against the Newton gradient, not its own
                    // right-hand side)
  const double* ggprev;   // [S] g'D^-1 g of the previous Newton iteration of the loop (<= 0:
                          // none) and the tolerance it was solved to: the forcing rule's
  const double* etaprev;  // inputs (scenes with SceneConst::forcing set)
  T *r, *z, *p0, *p1, *q;
  double* dx;
  const T* pinv;
  const int* drowptr;
  const int* dcol;
  const T* dval;
  T *P_pq, *P_rz0, *P_rz1, *P_gg;
  int* iters;
  int* indef;  // [S] set when PCG meets a direction of non-positive curvature (p.Ap <= 0)
  int max_iters;
  // coarse level (cg_on = 0: block Jacobi alone)
  int cg_on;
  int cg_mmax;                // largest coarse dimension of a scene (0 without the coarse level)
  const int* cg_blk_agg;      // [TN blocks] aggregate of the block, -1 if it has no soft node
  const int* cg_agg_b0;       // [aggregates] first TN block
  const int* cg_agg_b1;       // [aggregates] one past the last TN block
  const int* cg_sc_a0;        // [S] first aggregate of the scene
  const int* cg_sc_m;         // [S] coarse dimension (6 per aggregate)
  const long long* cg_sc_off; // [S] offset of the scene's inverse coarse operator
  const T* cg_d;              // [nodes][3] scaled rest offset from the aggregate centroid
  const T* cg_dw;             // [nodes][4] the same offset and a weight: 1 on the free soft
                              // nodes of an aggregate (whose offset is defined), else 0
  const float* cg_ainv;       // per scene m x m, row-major (FP32: preconditioner only)
  T* cg_rc;                   // [TN blocks][6] restricted residual partials (initial residual)
  const int* cg_sc_ts0;       // [S] first TS block of the scene's first aggregate
  const int* cg_sc_tsn;       // [S] TS blocks per aggregate (the last one may have fewer)
  const int* cg_sc_tsend;     // [S] one past the last TS block of the scene's aggregates
  T* P_qc;                    // [TS blocks][6] restriction of q = A p onto the rigid modes
  T *cg_rca0, *cg_rca1;       // [aggregates][6] restricted residual P^T r_k (by parity of k)
};
constexpr int kCoarseMaxAgg = 128;  // aggregates per scene (coarse dimension <= 768)

// Forcing term of inexact Newton (Eisenstat and Walker 1996, choice 2 with gamma = 0.9,
// alpha = 2 and its safeguard), on the preconditioned gradient norm: the relative PCG
// tolerance of the current Newton system given gg = g'D^-1 g now and at the previous
// iteration of the same Newton loop, and the previous tolerance; within [eta_min, kForcingMax].
constexpr double kForcingMax = 0.01;
__host__ __device__ inline double forcing_eta(double eta_min, double gg, double gg_prev, double eta_prev) {
  if (!(gg_prev > 0.0)) return fmax(kForcingMax, eta_min);
  double e = 0.9 * (gg / gg_prev);
  const double sg = 0.9 * eta_prev * eta_prev;
  if (sg > 0.1) e = fmax(e, sg);
  if (!(e >= eta_min)) e = eta_min;  // also when gg / gg_prev is not a number
  return fmin(e, fmax(kForcingMax, eta_min));
}
template <class T>
void launch_pcg_init(const View& V, const BlockTable& TN, const PcgBufsT<T>& B, hipStream_t s);
template <class T>
void launch_pcg_spmv(const View& V, const BlockTable& TN, const BlockTable& TS, const PcgBufsT<T>& B,
                     int parity, hipStream_t s);
template <class T>
void launch_pcg_coarse(const View& V, const BlockTable& TN, const PcgBufsT<T>& B, T* prz, hipStream_t s);
template <class T>
void launch_pcg_update(const View& V, const BlockTable& TN, const BlockTable& TS, const PcgBufsT<T>& B,
                       int parity, hipStream_t s);

// Process-wide kernel timing with HIP events (off by default).
struct Profiler {
  bool on = false;      // kernel timing with HIP events
  bool phases = false;  // host wall time per Newton-iteration phase
  double spmv_ms = 0.0;
  long long spmv_launches = 0;
  double spmv_bytes = 0.0;
  double pcg_ms = 0.0;        // wall time of the PCG chunk replays (after initialisation)
  long long pcg_iters = 0;    // iterations of those solves (largest per solve)
  long long refine_dirs = 0;    // Newton directions solved by FP32 passes (FP64_REFINED)
  long long refine_passes = 0;  // the FP32 passes they took
  // host wall time per Newton-iteration phase (each phase ends with a stream synchronisation
  // while profiling): candidates, derivatives + assembly, linear solve, convergence check,
  // swept candidates + CCD, line search + update
  static constexpr int kPhases = 6;
  double phase_ms[kPhases] = {0, 0, 0, 0, 0, 0};
  long long phase_calls = 0;
};
extern const char* const kPhaseNames[Profiler::kPhases];
Profiler& profiler();

// convergence, CCD, line search, update
void launch_pmax(const View& V, const double* p, unsigned long long* pmax, hipStream_t s);
// FP32 PCG with FP64 refinement (TACCEL_FP64_REFINED): FP32 copies of the FP64 system, the
// FP64 residual gres = g + H dx of the scenes still refining (pdone = 0; zero on fixed rows),
// its block-Jacobi norm and the gradient's per TN block (part[2 blk], part[2 blk + 1]), and
// dx = c (first pass) or dx += c (correction pass) on the scenes of the call (act).
void launch_to_f32(size_t n, const double* src, float* dst, hipStream_t s);
void launch_refine_resid(const View& V, const BlockTable& TS, const int* drowptr, const int* dcol,
                         const double* dval, const double* g, const double* dx, double* gres,
                         hipStream_t s);
void launch_refine_norm(const View& V, const BlockTable& TN, const double* pinv, const double* g,
                        const double* gres, double* part, hipStream_t s);
void launch_refine_apply(const View& V, const double* c, double* dx, int assign, hipStream_t s);
void launch_ccd(const View& V, int n, const int* cand_q, const int* cand_t,
                unsigned long long* amin, hipStream_t s);
void launch_scene_offsets(const View& V, int n, const int* cand_q, int* off, hipStream_t s);
// Friction pairs of the current step, lagged at its start (scene-contiguous): four contact
// vertex ids, closest-point weights, c0 = sum w_v x_v at the start, unit normal, mu lambda;
// soff [S+1] the first pair of each scene.
struct FricBufs {
  int n;
  int* v;        // [n][4]
  double* w;     // [n][4]
  double* c0;    // [n][3]
  double* nrm;   // [n][3]
  double* mul;   // [n]
  const int* soff;
};
void launch_fric_build(const View& V, int n, const int* pkind, const int* pv, const double* pmeps,
                       const FricBufs& F, hipStream_t s);
void launch_fric_derivs(const View& V, const FricBufs& F, int off, int* pv, double* pg, double* ph,
                        hipStream_t s);
void launch_debug_friction(int n, const int* kinds, const double* xn, const double* x,
                           const double* meps, double dhat, double kappa, double mu, double eh,
                           double* lam, double* e, double* g, double* H, hipStream_t s);

struct LsBufs {
  const double* p;        // node-space direction
  const double* abase;    // [S] largest trial step of this launch
  double* part_nodes;     // [node blocks][8]
  double* part_tets;      // [tet blocks][8]
  double* e_bodies;       // [Nb][9] energy at the current point, then at the 8 trials
  double* e_pairs;        // [ncand][9] same layout
  int* infeasible;        // [S] bit k: trial k hits J <= 0 or d <= 0
  const int* cand_off;    // [S+1]
  double* part_pairs;     // [pair blocks][8] sums of the pair energy differences
  double* dE;             // [S][8]
  FricBufs F;             // friction pairs (F.n = 0: none)
  double* e_fric;         // [F.n][9] like e_pairs
};
void launch_line_search(const View& V, const BlockTable& TN, const BlockTable& TT, const BlockTable& TP,
                        int ncand, const int* cand_q, const int* cand_t, const LsBufs& L, hipStream_t s);
void launch_update(const View& V, const double* p, const double* alpha, hipStream_t s);
void launch_al_apply(const View& V, const int* action, hipStream_t s);
void launch_body_reset(const View& V, double kappa0, hipStream_t s);
void launch_velocity(const View& V, const int* ok, hipStream_t s);
void launch_rollback(const View& V, const int* failed, hipStream_t s);
void launch_body_clear_lambda(const View& V, const int* flag, hipStream_t s);

// debug evaluators
void launch_debug_fem(int n, const double* x, const double* Dminv, const double* vol, double mu,
                      double lam, double* e, double* g, double* H, double* Hp, hipStream_t s);
void launch_debug_barrier(int n, const int* kinds, const double* x, const double* meps,
                          double dhat, double kappa, double* e, double* g, double* H, double* Hp,
                          int* types, hipStream_t s);
void launch_debug_ccd(int n, const int* kinds, const double* x, const double* p, double gap,
                      int max_iter, double* t, hipStream_t s);
void launch_debug_arap(int n, const double* A, double* e, double* g, double* H, double* Hp,
                       hipStream_t s);

}  // namespace tc
