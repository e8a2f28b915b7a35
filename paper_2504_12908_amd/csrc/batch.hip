// Host side of the batched IPC time step: scene setup (mesh topology, mass properties,
// sparsity pattern) and the per-step Newton / augmented-Lagrangian state machine.  All
// arithmetic of a step runs in the kernels of kernels.hip; the host only launches them,
// reads back a handful of per-scene flags and takes the control decisions.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <stdexcept>
#include <string>
#include <vector>

#include "coarse.h"
#include "kernels.h"
#include "prims.h"
#include "tactile.h"

namespace tc {

Profiler& profiler() {
  static Profiler p;
  return p;
}
const char* const kPhaseNames[Profiler::kPhases] = {"candidates", "derivatives", "solve",
                                                    "check", "ccd", "line_search"};

static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

struct ApiError : std::runtime_error {
  taccel_status st;
  ApiError(taccel_status s, const std::string& m) : std::runtime_error(m), st(s) {}
};

#define HIPCHECK(expr)                                                                  \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      throw ApiError(_e == hipErrorOutOfMemory ? TACCEL_ERR_OOM : TACCEL_ERR_HIP,       \
                     std::string(#expr) + ": " + hipGetErrorString(_e));                \
  } while (0)

// ------------------------------------------------------------------ device memory
struct Mem {
  taccel_runtime rt{};
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;   // second stream: contact Hessians
  hipStream_t side2 = nullptr;  // third stream: FEM and affine-body terms and their assembly
  bool own_stream = false;
  size_t held = 0;   // bytes allocated through this object and not yet released
  size_t limit = 0;  // 0: no limit; else an allocation that would pass it fails with OOM
  void* alloc(size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (limit && held + bytes > limit)
      throw ApiError(TACCEL_ERR_OOM, "device memory would exceed the object's limit of " +
                                         std::to_string(limit) + " bytes");
    void* p = nullptr;
    if (rt.alloc) {
      p = rt.alloc(bytes, rt.ctx);
      if (!p) throw ApiError(TACCEL_ERR_OOM, "runtime allocator returned NULL");
    } else {
      HIPCHECK(hipMalloc(&p, bytes));
    }
    held += bytes;
    return p;
  }
  void release(void* p, size_t bytes) {
    if (!p) return;
    held -= std::min(held, bytes);
    // work queued on either stream may still read the buffer
    if (stream) (void)hipStreamSynchronize(stream);
    if (side) (void)hipStreamSynchronize(side);
    if (side2) (void)hipStreamSynchronize(side2);
    if (rt.free) rt.free(p, rt.ctx);
    else (void)hipFree(p);
  }
};

template <class T>
struct DBuf {
  T* p = nullptr;
  size_t cap = 0;
  Mem* m = nullptr;
  void ensure(Mem* mem, size_t n) {
    m = mem;
    if (n <= cap && p) return;
    const size_t c = std::max<size_t>(n, cap + cap / 2);
    // the old buffer goes first; if the new allocation fails the object holds none
    if (p) m->release(p, sizeof(T) * std::max<size_t>(cap, 1));
    p = nullptr;
    cap = 0;
    p = static_cast<T*>(m->alloc(sizeof(T) * std::max<size_t>(c, 1)));
    cap = c;
  }
  // Copies h and waits for the copy: callers may pass temporaries.  (An asynchronous copy
  // from pageable memory may still be reading it after the call returns.)
  void upload(Mem* mem, const std::vector<T>& h) {
    ensure(mem, h.size());
    if (!h.empty()) {
      HIPCHECK(hipMemcpyAsync(p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, m->stream));
      HIPCHECK(hipStreamSynchronize(m->stream));
    }
  }
  void free() {
    if (p && m) m->release(p, sizeof(T) * std::max<size_t>(cap, 1));
    p = nullptr;
    cap = 0;
  }
};

// ------------------------------------------------------------------ host-side scene data
struct HostBody {
  int nv = 0, nf = 0;
  double com0[3] = {0, 0, 0};
  std::vector<double> xbar;  // [nv][3]
  bool prescribed = false;
  double r0 = 0, rprev = 0;
};
struct HostScene {
  int nv = 0, nb = 0, n_moving = 0;
  int node0 = 0, node1 = 0;
  std::vector<int> moving;  // internal soft vertex ids flagged 2, in the caller's vertex order
  std::vector<int> perm;    // caller's soft vertex id -> internal id (Morton order)
  std::vector<HostBody> bodies;
  std::vector<int> cv_world;  // world id per contact vertex of the scene
  int cv0 = 0, cv1 = 0, tri0 = 0, tri1 = 0, edge0 = 0, edge1 = 0;
  double stop = 0, h = 0;
  int max_newton = 100, max_al = 30, max_pcg = 10000;
};

// Volume integrals of 1, x, x x^T of a closed triangle mesh by the divergence theorem,
// reduced to per-face polynomial sums (Eberly, "Polyhedral Mass Properties").
static void polyhedron_integrals(const double* v, int nf, const int32_t* tris, double out[10]) {
  for (int k = 0; k < 10; ++k) out[k] = 0.0;
  auto sub = [](double w0, double w1, double w2, double& f1, double& f2, double& f3, double& g0,
                double& g1, double& g2) {
    const double t0 = w0 + w1;
    f1 = t0 + w2;
    const double t1 = w0 * w0;
    const double t2 = t1 + w1 * t0;
    f2 = t2 + w2 * f1;
    f3 = w0 * t1 + w1 * t2 + w2 * f2;
    g0 = f2 + w0 * (f1 + w0);
    g1 = f2 + w1 * (f1 + w1);
    g2 = f2 + w2 * (f1 + w2);
  };
  for (int f = 0; f < nf; ++f) {
    const double* p0 = v + 3 * tris[3 * f];
    const double* p1 = v + 3 * tris[3 * f + 1];
    const double* p2 = v + 3 * tris[3 * f + 2];
    const double a[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
    const double b[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
    const double d[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    double f1x, f2x, f3x, g0x, g1x, g2x, f1y, f2y, f3y, g0y, g1y, g2y, f1z, f2z, f3z, g0z, g1z, g2z;
    sub(p0[0], p1[0], p2[0], f1x, f2x, f3x, g0x, g1x, g2x);
    sub(p0[1], p1[1], p2[1], f1y, f2y, f3y, g0y, g1y, g2y);
    sub(p0[2], p1[2], p2[2], f1z, f2z, f3z, g0z, g1z, g2z);
    out[0] += d[0] * f1x;
    out[1] += d[0] * f2x;
    out[2] += d[1] * f2y;
    out[3] += d[2] * f2z;
    out[4] += d[0] * f3x;
    out[5] += d[1] * f3y;
    out[6] += d[2] * f3z;
    out[7] += d[0] * (p0[1] * g0x + p1[1] * g1x + p2[1] * g2x);
    out[8] += d[1] * (p0[2] * g0y + p1[2] * g1y + p2[2] * g2y);
    out[9] += d[2] * (p0[0] * g0z + p1[0] * g1z + p2[0] * g2z);
  }
  out[0] /= 6.0;
  for (int k = 1; k < 4; ++k) out[k] /= 24.0;
  for (int k = 4; k < 7; ++k) out[k] /= 60.0;
  for (int k = 7; k < 10; ++k) out[k] /= 120.0;
}

static void inverse3(const double* A, double* out) {
  const double c0 = A[4] * A[8] - A[5] * A[7], c1 = A[5] * A[6] - A[3] * A[8], c2 = A[3] * A[7] - A[4] * A[6];
  const double det = A[0] * c0 + A[1] * c1 + A[2] * c2;
  out[0] = c0 / det;
  out[1] = (A[2] * A[7] - A[1] * A[8]) / det;
  out[2] = (A[1] * A[5] - A[2] * A[4]) / det;
  out[3] = c1 / det;
  out[4] = (A[0] * A[8] - A[2] * A[6]) / det;
  out[5] = (A[2] * A[3] - A[0] * A[5]) / det;
  out[6] = c2 / det;
  out[7] = (A[1] * A[6] - A[0] * A[7]) / det;
  out[8] = (A[0] * A[4] - A[1] * A[3]) / det;
}

// ------------------------------------------------------------------ implementation
struct Batch::Impl {
  Mem mem;
  int S = 0, Nn = 0, Nt = 0, Nb = 0, Ncv = 0, Ntr = 0, Ned = 0, Nq = 0, nnz = 0;
  std::vector<HostScene> hs;
  std::vector<SceneConst> hsc;
  std::vector<int> h_ntype, h_nscene, h_bnode, h_bscene, h_bpres;
  std::vector<double> spmv_static_blocks;  // per scene: stored blocks of free rows
  std::vector<double> spmv_free_nodes;
  std::vector<hipEvent_t> ev_pool;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_join2 = nullptr;
  // static device data
  DBuf<SceneConst> d_sc;
  DBuf<double> x, xn, xhat, v, mass;
  DBuf<int> nfree, nscene, nbody, ntype;
  DBuf<int> tv, tscene;
  DBuf<double> Dminv, tvol;
  DBuf<int> rowptr, col, diag, vptr, vlist;
  DBuf<double> val;
  DBuf<int> bnode, bscene, bpres, bsnap, bcv0, bcv1;
  DBuf<double> bmass, bvol, bstar, blam, bkap, bgrad, bhess, bpinv;
  DBuf<int> cvn, cvb, cvfix, cvscene, cvworld, trv, edv, qkind, qidx, qscene;
  DBuf<double> cvx, cpos, cdisp, cend, elen2;
  DBuf<int> act, pdone, exact, indef;
  // per scene, the previous Newton iteration of its current loop: step size and max vertex
  // displacement of the direction (they decide whether this iteration uses exact Hessians)
  std::vector<double> prev_alpha, prev_pmax;
  // forcing terms (scenes with pcg_forcing): g'D^-1 g of the previous Newton iteration of the
  // loop (-1 at a loop's start) and its tolerance, uploaded before every solve; the block
  // partials of g'D^-1 g read back after it
  std::vector<double> gg_prev_h, eta_prev_h;
  DBuf<double> fg_prev;  // [2 S]: gg_prev, eta_prev
  std::vector<double> ggd_h;
  std::vector<float> ggf_h;
  void gg_readback() {  // enqueued; valid after the next sync()
    const size_t nb = (size_t)TN.nblk;
    if (nb == 0) return;
    if (mixed || refine) {
      ggf_h.resize(nb);
      d2h(ggf_h.data(), reinterpret_cast<const float*>(P_gg.p), nb);
    } else {
      ggd_h.resize(nb);
      d2h(ggd_h.data(), P_gg.p, nb);
    }
  }
  double gg_scene(int k) const {  // block order: the same sum on every call
    double acc = 0.0;
    for (int b = tn_sblk_host[k]; b < tn_sblk_host[k + 1]; ++b)
      acc += (mixed || refine) ? (double)ggf_h[b] : ggd_h[b];
    return acc;
  }
  // the tolerance the solve of scene k used (after gg_readback and its sync)
  double eta_used(int k) const {
    return hsc[k].forcing ? forcing_eta(hsc[k].pcg_eta, gg_scene(k), gg_prev_h[k], eta_prev_h[k])
                          : hsc[k].pcg_eta;
  }
  std::vector<int> exact_h;
  // block tables
  DBuf<int> tn_sc, tn_b0, tn_b1, tn_sblk, tt_sc, tt_b0, tt_b1, tt_sblk, ts_sc, ts_b0, ts_b1, ts_sblk;
  BlockTable TN, TT, TS;
  // candidate list that covers every pair that can be closer than dhat at the current
  // positions (the swept set of the last Newton iteration, valid until something moves
  // outside its sweep)
  bool cover_valid = false;
  int n_cover = 0;
  bool device_touched = false;
  bool xn_valid = false;       // xn holds the positions at the start of the current step
  std::vector<int> act_host;   // host copy of act for the current Newton iteration
  int pcg_last_max = 0;        // largest PCG iteration count of the previous solve
  std::vector<taccel_step_stats> last_stats;  // per scene: statistics of its last step
  bool validate_only = false;  // build() stops after the host-side checks
  int mixed = 0;  // 1: FP32 Hessian blocks, assembly, SpMV and PCG (taccel_precision MIXED)
  // 1: FP64 system, FP32 PCG passes with FP64 refinement (taccel_precision FP64_REFINED)
  int refine = 0;
  static constexpr int kRefinePasses = 3;  // FP32 solves per Newton direction, at most
  // FP32 copies of the FP64 system for the passes, the FP32 coarse offsets, the correction of
  // a pass, the FP64 residual and its per-block norms
  DBuf<float> val32, dval32, pinv32, bpinv32, cg_d32, cg_dw32;
  DBuf<double> dxc, gres, rpart;
  int nh_last = 0;  // contact and body block records of the current Newton system
  std::vector<int> tn_sblk_host;  // [S + 1] first TN block of each scene
  std::vector<int> solve_refined(const View& V, const int* nseg_d, const std::vector<int>& act_s);
  // dynamic work buffers
  BroadPhase bp;
  DBuf<double> bp_tbox;
  DBuf<int> bp_tcell, bp_tncell, bp_toff, bp_bcount, bp_bstart, bp_bfill, bp_qcount, bp_qoff;
  DBuf<BpEntry> bp_entries;
  DBuf<int> cq, ct, sq, st, cflag, cpos_idx;
  DBuf<int> pkind, pv, pscene;
  DBuf<double> pmeps, pg, ph;
  DBuf<int> hcnt, gcnt, hoff, goff, hidx, gidx, hsrc, gsrc, hidx2, gidx2;
  DBuf<uint64_t> hkey, gkey, hkey2, gkey2;
  DBuf<double> hcoef, gcoef;
  DBuf<int> sflag, segid, segstart, drow, dcol, rowcnt, drowptr;
  DBuf<double> dval;
  DBuf<double> g, r, z, p, p1, q, dx, pinv;
  DBuf<double> P_pq, P_rz0, P_rz1, P_gg;
  // two-level preconditioner: coarse space of 6 rigid modes per aggregate of 64-node
  // blocks, with the inverse of its rest-state operator per scene
  DBuf<int> cg_blk_agg, cg_agg_b0, cg_agg_b1, cg_sc_a0, cg_sc_m;
  DBuf<long long> cg_sc_off;
  DBuf<double> cg_d, cg_ainv, cg_rc;  // cg_d, cg_rc: T-typed storage; cg_ainv: float
  DBuf<double> P_qc, cg_rca0, cg_rca1, cg_dw;  // T-typed storage
  DBuf<int> cg_sc_ts0, cg_sc_tsn, cg_sc_tsend;
  DBuf<int> bp_tmp;  // broad phase: candidates in emitted order before the per-query sort
  int cg_on = 0;
  int cg_mmax = 0;  // largest coarse dimension of a scene
  DBuf<int> iters, bad, infeasible, scnt, cand_off, action, okflag, failflag, snapcand;
  DBuf<unsigned long long> u64s;  // pmax [S], amin [S], body residuals [Nb]
  DBuf<double> abase, alpha, dE, part_nodes, part_tets, e_bodies, e_pairs, part_pairs;
  // friction pairs of the current step, lagged at its start (scene-contiguous)
  bool any_fric = false;
  int nfric = 0;
  DBuf<int> fv, fsoff;
  DBuf<double> fw, fc0, fnrm, fmul, e_fric;
  FricBufs fric_bufs() {
    FricBufs F;
    F.n = nfric;
    F.v = fv.p;
    F.w = fw.p;
    F.c0 = fc0.p;
    F.nrm = fnrm.p;
    F.mul = fmul.p;
    F.soff = fsoff.p;
    return F;
  }
  void build_friction(const int* mask);
  std::vector<int32_t> contacts(int k);
  int prepare_pairs(std::vector<int>& bp_bad);
  int* derivatives(int np, int npf);
  void begin_step(const taccel_targets* tg, const int* mask, std::vector<int>& infeasible_target,
                  std::vector<char>& snapped_host);
  // tactile outputs: rest positions of every node and work buffers
  DBuf<double> xrest, tac_bary, tac_pos, tac_flow, tac_depth, tac_normal;
  DBuf<int> tac_nodes, tac_zidx;
  DBuf<unsigned long long> tac_zkey;
  // caller's soft vertex ids of scene k -> node ids (checked)
  std::vector<int> soft_nodes(int k, int n, const int32_t* ids) const {
    const HostScene& H = hs[k];
    std::vector<int> out(n);
    for (int i = 0; i < n; ++i) {
      if (ids[i] < 0 || ids[i] >= H.nv) throw ApiError(TACCEL_ERR_ARG, "soft vertex id out of range");
      out[i] = H.node0 + H.perm[ids[i]];
    }
    return out;
  }
  // swept candidates in blocks of one scene (line-search partial sums), rebuilt per iteration
  static constexpr int kPairChunk = 1024;
  std::vector<int> tp_sc_h, tp_c0_h, tp_c1_h, tp_sblk_h;
  DBuf<int> tp_sc, tp_b0, tp_b1, tp_sblk;
  BlockTable TP;
  DBuf<int> scalars;  // device scalars for scan totals
  DBuf<char> scratch;
  DBuf<int> mv_nodes;
  DBuf<double> mv_tgt;
  // Pinned host staging for small transfers.  A readback is copied into it asynchronously
  // and reaches its destination in sync(); an upload is copied into it and read by the device
  // before the next sync(), which makes the whole area free again.  Transfers that do not
  // fit go through pageable memory (synchronous).
  char* h_pin = nullptr;
  size_t h_pin_bytes = 0, h_pin_used = 0;
  struct Readback {
    void* dst;
    const void* staged;
    size_t bytes;
  };
  std::vector<Readback> readbacks;
  static constexpr size_t kStageBytes = 4u << 20, kStageMaxCopy = 256u << 10;
  void* stage_take(size_t bytes) {
    if (!h_pin || bytes > kStageMaxCopy) return nullptr;
    const size_t at = (h_pin_used + 255) & ~size_t(255);
    if (at + bytes > h_pin_bytes) return nullptr;
    h_pin_used = at + bytes;
    return h_pin + at;
  }
  // readbacks whose destinations may no longer exist (an error unwound their callers)
  void discard_pending() {
    readbacks.clear();
    h_pin_used = 0;
  }

  View view() const {
    View V;
    V.S = S; V.Nn = Nn; V.Nt = Nt; V.Nb = Nb; V.Ncv = Ncv; V.Ntr = Ntr; V.Ned = Ned; V.Nq = Nq;
    V.sc = d_sc.p;
    V.x = x.p; V.xrest = xrest.p; V.xn = xn.p; V.xhat = xhat.p; V.v = v.p; V.mass = mass.p;
    V.nfree = nfree.p; V.nscene = nscene.p; V.nbody = nbody.p; V.ntype = ntype.p;
    V.tv = tv.p; V.Dminv = Dminv.p; V.tvol = tvol.p; V.tscene = tscene.p;
    V.rowptr = rowptr.p; V.col = col.p; V.val = val.p; V.diag = diag.p;
    V.vptr = vptr.p; V.vlist = vlist.p;
    V.bnode = bnode.p; V.bscene = bscene.p; V.bmass = bmass.p; V.bvol = bvol.p; V.bpres = bpres.p;
    V.bstar = bstar.p; V.blam = blam.p; V.bkap = bkap.p; V.bsnap = bsnap.p; V.bgrad = bgrad.p;
    V.bhess = bhess.p; V.bpinv = bpinv.p; V.bcv0 = bcv0.p; V.bcv1 = bcv1.p;
    V.cvn = cvn.p; V.cvb = cvb.p; V.cvx = cvx.p; V.cvfix = cvfix.p; V.cvscene = cvscene.p;
    V.cvworld = cvworld.p; V.cpos = cpos.p; V.cdisp = cdisp.p; V.trv = trv.p; V.edv = edv.p;
    V.elen2 = elen2.p; V.qkind = qkind.p; V.qidx = qidx.p; V.qscene = qscene.p;
    V.act = act.p; V.pdone = pdone.p; V.exact = exact.p;
    return V;
  }

  hipStream_t stream() const { return mem.stream; }
  void sync() {
    const hipError_t e = hipStreamSynchronize(mem.stream);
    // the destinations are alive here (their owners are waiting in this call)
    for (const Readback& r : readbacks) std::memcpy(r.dst, r.staged, r.bytes);
    readbacks.clear();
    h_pin_used = 0;
    HIPCHECK(e);
  }
  template <class T>
  void d2h(T* dst, const T* src, size_t n) {
    if (!n) return;
    const size_t bytes = sizeof(T) * n;
    if (void* st = stage_take(bytes)) {
      HIPCHECK(hipMemcpyAsync(st, src, bytes, hipMemcpyDeviceToHost, mem.stream));
      readbacks.push_back({dst, st, bytes});
    } else {
      HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, mem.stream));
    }
  }
  template <class T>
  void h2d(T* dst, const T* src, size_t n) {
    if (!n) return;
    const size_t bytes = sizeof(T) * n;
    if (void* st = stage_take(bytes)) {
      std::memcpy(st, src, bytes);
      HIPCHECK(hipMemcpyAsync(dst, st, bytes, hipMemcpyHostToDevice, mem.stream));
    } else {
      // pageable source: wait for the copy, so the caller may release it at once
      HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, mem.stream));
      HIPCHECK(hipStreamSynchronize(mem.stream));
    }
  }
  void zero(void* p, size_t bytes) {
    if (bytes) HIPCHECK(hipMemsetAsync(p, 0, bytes, mem.stream));
  }
  int read_int(const int* d) {
    int v = 0;
    d2h(&v, d, 1);
    sync();
    return v;
  }
  void ensure_scratch(size_t bytes) { scratch.ensure(&mem, bytes); }
  int scan(const int* in, int* out, int n) {
    scan_async(in, out, n, scalars.p);
    return read_int(scalars.p);
  }
  // exclusive scan whose total stays on the device
  void scan_async(const int* in, int* out, int n, int* total) {
    ensure_scratch(scan_scratch_bytes(n));
    HIPCHECK(exclusive_scan(in, out, n, total, scratch.p, mem.stream));
  }
  void sort(uint64_t* keys, int* vals, uint64_t* tk, int* tv_, int n, int bits) {
    ensure_scratch(sort_scratch_bytes(n));
    HIPCHECK(radix_sort_pairs(keys, vals, tk, tv_, n, bits, scratch.p, mem.stream));
  }

  // PCG chunks replayed as a HIP graph (16 iterations = 32 kernels); re-captured when a
  // buffer it reads is reallocated or profiling is switched
  // the graphs the executable was instantiated from or updated with: kept until the
  // executable itself is destroyed (a tool that traces graph launches may still refer to
  // the nodes it was built from)
  std::vector<hipGraph_t> pcg_graphs;
  hipGraphExec_t pcg_exec = nullptr;
  std::vector<const void*> pcg_key;
  static constexpr int kPcgChunk = 16;
  template <class T>
  void run_pcg(const View& V, const PcgBufsT<T>& B, const int* nseg_d);
  template <class T>
  PcgBufsT<T> pcg_bufs();
  void build(const taccel_scene_desc* d, int n);
  // ovf (nullable): per-scene flags of boxes spanning too many cells (exploded positions or
  // a runaway direction); without it such a scene makes the call throw TACCEL_NAN
  int broad_phase(const double* P0, const double* P1, int all, DBuf<int>& oq, DBuf<int>& ot,
                  std::vector<int>* ovf = nullptr);
  DBuf<int> bp_ovf;
  void newton_iteration(std::vector<int>& last, std::vector<int>& ls_fail, std::vector<int>& nan_,
                        std::vector<int>& pcg_it, std::vector<int>& n_active, std::vector<int>& halvings);
  taccel_status step(const taccel_targets* t, taccel_status* per_scene, taccel_step_stats* st,
                     const int* mask);
  size_t device_bytes() const;
  void release_all();
};

// Order of n points along a Morton (Z-order) curve of their bounding box, 10 bits per axis;
// ties keep the input order.  Returns perm with perm[i] = rank of point i.
static std::vector<int> morton_order(const double* X, int n) {
  std::vector<int> perm(n);
  if (n == 0) return perm;
  double lo[3], hi[3];
  for (int c = 0; c < 3; ++c) lo[c] = hi[c] = X[c];
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) {
      lo[c] = std::min(lo[c], X[3 * (size_t)i + c]);
      hi[c] = std::max(hi[c], X[3 * (size_t)i + c]);
    }
  std::vector<std::pair<uint32_t, int>> key(n);
  for (int i = 0; i < n; ++i) {
    uint32_t q[3];
    for (int c = 0; c < 3; ++c) {
      const double span = hi[c] - lo[c];
      const double t = span > 0.0 ? (X[3 * (size_t)i + c] - lo[c]) / span : 0.0;
      q[c] = (uint32_t)std::min(1023.0, std::max(0.0, std::floor(t * 1024.0)));
    }
    uint32_t k = 0;
    for (int b = 9; b >= 0; --b)
      for (int c = 2; c >= 0; --c) k = (k << 1) | ((q[c] >> b) & 1u);
    key[i] = {k, i};
  }
  std::sort(key.begin(), key.end());
  for (int r = 0; r < n; ++r) perm[key[r].second] = r;
  return perm;
}

static int bits_for(uint64_t v) {
  int b = 1;
  while (b < 64 && (v >> b) != 0) ++b;
  return b;
}

// ------------------------------------------------------------------ setup
void Batch::Impl::build(const taccel_scene_desc* descs, int n) {
  S = n;
  hs.resize(S);
  hsc.resize(S);
  last_stats.assign(S, taccel_step_stats{});
  prev_alpha.assign(S, 0.0);
  prev_pmax.assign(S, 0.0);
  gg_prev_h.assign(S, -1.0);
  eta_prev_h.assign(S, 0.0);
  exact_h.assign(S, 0);
  std::vector<double> h_x, h_mass, h_Dminv_aos, h_tvol;
  std::vector<int> h_nfree, h_nbody, h_tv_aos, h_tscene;
  std::vector<int> h_bcv0, h_bcv1;
  std::vector<double> h_bmass, h_bvol;
  std::vector<int> h_cvn, h_cvb, h_cvfix, h_cvscene, h_cvworld, h_trv, h_edv, h_qkind, h_qidx, h_qscene;
  std::vector<double> h_cvx, h_elen2;
  std::vector<int> tn_sc_h, tn_b0_h, tn_b1_h, tn_sblk_h, tt_sc_h, tt_b0_h, tt_b1_h, tt_sblk_h;
  std::vector<int> ts_sc_h, ts_b0_h, ts_b1_h, ts_sblk_h;
  // static BSR built per scene and concatenated
  std::vector<int> h_rowptr(1, 0), h_col, h_diag, h_vptr(1, 0), h_vlist;
  for (int s = 0; s < S; ++s) {
    const taccel_scene_desc& du = descs[s];  // caller's vertex order
    HostScene& H = hs[s];
    const taccel_params& P = du.params;
    if (!(P.h > 0) || !(P.dhat > 0) || !(P.kappa >= 0) || !(P.newton_tol > 0))
      throw ApiError(TACCEL_ERR_ARG, "scene " + std::to_string(s) + ": h, dhat, newton_tol must be > 0");
    const int nv = du.soft.nv, nt = du.soft.nt, nb = du.n_bodies;
    if (nv < 0 || nt < 0 || nb < 0 || (nv > 0 && !du.soft.verts) || (nt > 0 && !du.soft.tets) ||
        (nb > 0 && !du.bodies))
      throw ApiError(TACCEL_ERR_ARG, "scene " + std::to_string(s) + ": bad soft/body sizes");
    // ---- internal vertex order: soft vertices sorted along a Morton curve of their rest
    // positions, so consecutive nodes (each 64-node block in particular) are spatially
    // compact; tets keep their order and refer to the new ids
    for (int k = 0; k < 4 * nt; ++k)
      if (du.soft.tets[k] < 0 || du.soft.tets[k] >= nv) throw ApiError(TACCEL_ERR_ARG, "tet index out of range");
    if (du.soft.dirichlet)
      for (int i = 0; i < nv; ++i)
        if (du.soft.dirichlet[i] > 2) throw ApiError(TACCEL_ERR_ARG, "dirichlet flag must be 0, 1 or 2");
    H.perm = morton_order(du.soft.verts, nv);
    std::vector<double> pverts(3 * (size_t)nv);
    std::vector<int32_t> ptets(4 * (size_t)nt);
    std::vector<uint8_t> pdir(du.soft.dirichlet ? nv : 0);
    std::vector<int> iperm(nv);
    for (int i = 0; i < nv; ++i) {
      iperm[H.perm[i]] = i;
      for (int c = 0; c < 3; ++c) pverts[3 * (size_t)H.perm[i] + c] = du.soft.verts[3 * (size_t)i + c];
      if (du.soft.dirichlet) pdir[H.perm[i]] = du.soft.dirichlet[i];
    }
    for (int k = 0; k < 4 * nt; ++k) ptets[k] = H.perm[du.soft.tets[k]];
    taccel_scene_desc d = du;
    d.soft.verts = pverts.data();
    d.soft.tets = ptets.data();
    d.soft.dirichlet = du.soft.dirichlet ? pdir.data() : nullptr;
    H.nv = nv;
    H.nb = nb;
    H.h = P.h;
    H.max_newton = P.max_newton > 0 ? P.max_newton : 100;
    H.max_al = P.max_al > 0 ? P.max_al : 30;
    H.max_pcg = P.max_pcg > 0 ? P.max_pcg : 10000;
    SceneConst& C = hsc[s];
    std::memset(&C, 0, sizeof(C));
    C.h = P.h;
    C.dhat = P.dhat;
    C.kappa = P.kappa;
    C.kappa_s = P.kappa_s;
    C.mu = d.soft.youngs / (2.0 * (1.0 + d.soft.poisson));
    C.lam = d.soft.youngs * d.soft.poisson / ((1.0 + d.soft.poisson) * (1.0 - 2.0 * d.soft.poisson));
    C.pcg_eta = P.pcg_eta > 0 ? P.pcg_eta : (P.precision == TACCEL_MIXED ? 1e-3 : 1e-4);
    for (int c = 0; c < 3; ++c) C.grav[c] = P.gravity[c];
    if (!(P.friction >= 0.0) || (P.friction > 0.0 && !(P.eps_v > 0.0)))
      throw ApiError(TACCEL_ERR_ARG, "friction must be >= 0, with eps_v > 0 when friction > 0");
    C.fmu = P.friction;
    C.eh = P.eps_v * P.h;
    if (C.fmu > 0.0) any_fric = true;
    C.precision = P.precision;
    if (P.pcg_forcing != 0 && P.pcg_forcing != 1)
      throw ApiError(TACCEL_ERR_ARG, "pcg_forcing must be 0 or 1");
    C.forcing = P.pcg_forcing;
    if (P.precision != TACCEL_FP64 && P.precision != TACCEL_MIXED && P.precision != TACCEL_FP64_REFINED)
      throw ApiError(TACCEL_ERR_ARG, "precision must be TACCEL_FP64, TACCEL_MIXED or TACCEL_FP64_REFINED");
    if (s == 0) {
      mixed = P.precision == TACCEL_MIXED;
      refine = P.precision == TACCEL_FP64_REFINED;
    } else if (mixed != (P.precision == TACCEL_MIXED) || refine != (P.precision == TACCEL_FP64_REFINED)) {
      throw ApiError(TACCEL_ERR_ARG, "all scenes of a batch must use the same precision");
    }
    // A 256-scene mixed-precision batch ended in a GPU memory fault whose cause is not shown;
    // until it is, mixed precision runs one scene per object.  (The host build of the tests
    // defines TACCEL_HOST_MIXED_BATCHES to run such batches under its guard pages.)
#ifndef TACCEL_HOST_MIXED_BATCHES
    if (mixed && n > 1)
      throw ApiError(TACCEL_ERR_ARG, "mixed precision is limited to one scene per batch");
#endif
    // ---- nodes
    const int node0 = Nn;
    H.node0 = node0;
    const int n_soft_pad = (nv + 3) / 4 * 4;
    const int nn = n_soft_pad + 4 * nb;
    C.node0 = node0;
    C.node1 = node0 + nn;
    H.node1 = C.node1;
    h_x.resize(3 * (size_t)(node0 + nn), 0.0);
    h_mass.resize(node0 + nn, 0.0);
    h_nfree.resize(node0 + nn, 0);
    h_nbody.resize(node0 + nn, -1);
    h_ntype.resize(node0 + nn, 3);
    h_nscene.resize(node0 + nn, s);
    for (int i = 0; i < nv; ++i) {
      for (int c = 0; c < 3; ++c) h_x[3 * (size_t)(node0 + i) + c] = d.soft.verts[3 * i + c];
      const int flag = d.soft.dirichlet ? d.soft.dirichlet[i] : 0;
      if (flag > 2) throw ApiError(TACCEL_ERR_ARG, "dirichlet flag must be 0, 1 or 2");
      h_nfree[node0 + i] = flag == 0;
      h_ntype[node0 + i] = 0;
    }
    for (int u = 0; u < nv; ++u)
      if (du.soft.dirichlet && du.soft.dirichlet[u] == 2) H.moving.push_back(H.perm[u]);
    H.n_moving = (int)H.moving.size();
    // ---- tets
    const int tet0 = Nt;
    C.tet0 = tet0;
    C.tet1 = tet0 + nt;
    std::vector<std::vector<int>> adj(nv);
    std::vector<std::vector<int>> inc(nv);  // tet*4 + a (global tet ids)
    for (int e = 0; e < nt; ++e) {
      int t[4];
      for (int a = 0; a < 4; ++a) {
        t[a] = d.soft.tets[4 * e + a];
        if (t[a] < 0 || t[a] >= nv) throw ApiError(TACCEL_ERR_ARG, "tet index out of range");
      }
      double Dm[9];
      for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) Dm[3 * i + k] = d.soft.verts[3 * t[k + 1] + i] - d.soft.verts[3 * t[0] + i];
      const double det = Dm[0] * (Dm[4] * Dm[8] - Dm[5] * Dm[7]) - Dm[1] * (Dm[3] * Dm[8] - Dm[5] * Dm[6]) +
                         Dm[2] * (Dm[3] * Dm[7] - Dm[4] * Dm[6]);
      if (!(det > 0.0)) throw ApiError(TACCEL_ERR_ARG, "inverted or degenerate tet " + std::to_string(e));
      double Di[9];
      inverse3(Dm, Di);
      for (int k = 0; k < 9; ++k) h_Dminv_aos.push_back(Di[k]);
      const double vol = det / 6.0;
      h_tvol.push_back(vol);
      for (int a = 0; a < 4; ++a) {
        h_tv_aos.push_back(node0 + t[a]);
        h_mass[node0 + t[a]] += d.soft.density * vol / 4.0;
        inc[t[a]].push_back(4 * (tet0 + e) + a);
        for (int b = 0; b < 4; ++b) adj[t[a]].push_back(t[b]);
      }
      h_tscene.push_back(s);
    }
    // static BSR rows for every node of the scene (soft rows carry the FEM pattern)
    for (int i = 0; i < nn; ++i) {
      const int node = node0 + i;
      if (i < nv) {
        std::vector<int>& a = adj[i];
        a.push_back(i);
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
        int dpos = -1;
        for (int j : a) {
          if (j == i) dpos = (int)h_col.size();
          h_col.push_back(node0 + j);
        }
        h_diag.push_back(dpos);
        for (int code : inc[i]) h_vlist.push_back(code);
      } else {
        h_diag.push_back(-1);
      }
      h_rowptr.push_back((int)h_col.size());
      h_vptr.push_back((int)h_vlist.size());
    }
    // ---- contact surface: boundary faces of the tet mesh
    struct Face { int k[3]; int o[3]; };
    std::vector<Face> faces;
    faces.reserve(4 * (size_t)nt);
    for (int e = 0; e < nt; ++e) {
      const int* t = d.soft.tets + 4 * e;
      const int f[4][3] = {{t[1], t[2], t[3]}, {t[0], t[3], t[2]}, {t[0], t[1], t[3]}, {t[0], t[2], t[1]}};
      for (int k = 0; k < 4; ++k) {
        Face F;
        for (int j = 0; j < 3; ++j) F.o[j] = F.k[j] = f[k][j];
        std::sort(F.k, F.k + 3);
        faces.push_back(F);
      }
    }
    std::sort(faces.begin(), faces.end(), [](const Face& a, const Face& b) {
      return std::lexicographical_compare(a.k, a.k + 3, b.k, b.k + 3);
    });
    std::vector<std::array<int, 3>> bfaces;
    for (size_t i = 0; i < faces.size();) {
      size_t j = i + 1;
      while (j < faces.size() && std::equal(faces[i].k, faces[i].k + 3, faces[j].k)) ++j;
      if (j - i == 1) bfaces.push_back({faces[i].o[0], faces[i].o[1], faces[i].o[2]});
      else if (j - i > 2) throw ApiError(TACCEL_ERR_ARG, "non-manifold tet mesh (face shared by >2 tets)");
      i = j;
    }
    std::vector<int> soft_cv(nv, -1);
    for (const auto& f : bfaces)
      for (int k = 0; k < 3; ++k) soft_cv[f[k]] = 0;
    const int cv0 = Ncv;
    H.cv0 = cv0;
    int ncv = 0;
    for (int i = 0; i < nv; ++i)
      if (soft_cv[i] == 0) {
        soft_cv[i] = cv0 + ncv++;
        h_cvn.push_back(node0 + i);
        h_cvb.push_back(-1);
        for (int c = 0; c < 3; ++c) h_cvx.push_back(0.0);
        const int flag = d.soft.dirichlet ? d.soft.dirichlet[i] : 0;
        h_cvfix.push_back(flag == 1);
        h_cvscene.push_back(s);
        h_cvworld.push_back(iperm[i]);
        H.cv_world.push_back(iperm[i]);
      }
    std::vector<std::array<int, 3>> tris;
    for (const auto& f : bfaces) tris.push_back({soft_cv[f[0]], soft_cv[f[1]], soft_cv[f[2]]});
    // ---- affine bodies
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = 0; i < nv; ++i)
      for (int c = 0; c < 3; ++c) {
        lo[c] = std::min(lo[c], d.soft.verts[3 * i + c]);
        hi[c] = std::max(hi[c], d.soft.verts[3 * i + c]);
      }
    C.body0 = Nb;
    int world = nv;
    for (int b = 0; b < nb; ++b) {
      const taccel_body_desc& B = d.bodies[b];
      if (B.nv < 4 || B.nf < 4 || !B.verts || !B.tris || !(B.density > 0))
        throw ApiError(TACCEL_ERR_ARG, "affine body needs >= 4 vertices, >= 4 faces, density > 0");
      for (int k = 0; k < 3 * B.nf; ++k)
        if (B.tris[k] < 0 || B.tris[k] >= B.nv) throw ApiError(TACCEL_ERR_ARG, "body triangle index out of range");
      double I[10];
      polyhedron_integrals(B.verts, B.nf, B.tris, I);
      const double vol = I[0];
      if (!(vol > 0.0)) throw ApiError(TACCEL_ERR_ARG, "affine body encloses no positive volume");
      HostBody hb;
      hb.nv = B.nv;
      hb.nf = B.nf;
      hb.prescribed = B.prescribed != 0;
      for (int c = 0; c < 3; ++c) hb.com0[c] = I[1 + c] / vol;
      const double sm[9] = {I[4], I[7], I[9], I[7], I[5], I[8], I[9], I[8], I[6]};
      h_bmass.push_back(B.density * vol);
      for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) h_bmass.push_back(B.density * (sm[3 * a + c] - vol * hb.com0[a] * hb.com0[c]));
      h_bvol.push_back(vol);
      const int bn = node0 + n_soft_pad + 4 * b;
      h_bnode.push_back(bn);
      h_bscene.push_back(s);
      h_bpres.push_back(hb.prescribed);
      for (int u = 0; u < 4; ++u) {
        h_nbody[bn + u] = Nb + b;
        h_ntype[bn + u] = u == 0 ? 1 : 2;
        h_nfree[bn + u] = 1;
      }
      for (int c = 0; c < 3; ++c) {
        h_x[3 * (size_t)bn + c] = hb.com0[c];
        h_x[3 * (size_t)(bn + 1 + c) + c] = 1.0;
      }
      const int bcv = cv0 + ncv;
      h_bcv0.push_back(bcv);
      for (int k = 0; k < B.nv; ++k) {
        for (int c = 0; c < 3; ++c) {
          const double xb = B.verts[3 * k + c] - hb.com0[c];
          hb.xbar.push_back(xb);
          h_cvx.push_back(xb);
          lo[c] = std::min(lo[c], B.verts[3 * k + c]);
          hi[c] = std::max(hi[c], B.verts[3 * k + c]);
        }
        h_cvn.push_back(-1);
        h_cvb.push_back(Nb + b);
        h_cvfix.push_back(0);
        h_cvscene.push_back(s);
        h_cvworld.push_back(world + k);
        H.cv_world.push_back(world + k);
      }
      for (int f = 0; f < B.nf; ++f)
        tris.push_back({bcv + B.tris[3 * f], bcv + B.tris[3 * f + 1], bcv + B.tris[3 * f + 2]});
      ncv += B.nv;
      world += B.nv;
      h_bcv1.push_back(cv0 + ncv);
      H.bodies.push_back(hb);
    }
    C.body1 = Nb + nb;
    C.cv0 = cv0;
    C.cv1 = cv0 + ncv;
    H.cv1 = C.cv1;
    // rest positions of contact vertices (for edge rest lengths)
    auto rest_pos = [&](int cv, double* p) {
      const int li = cv - cv0;
      const int w = H.cv_world[li];
      if (w < nv) {
        for (int c = 0; c < 3; ++c) p[c] = du.soft.verts[3 * w + c];
      } else {
        int off = nv;
        for (int b = 0; b < nb; ++b) {
          if (w < off + d.bodies[b].nv) {
            for (int c = 0; c < 3; ++c) p[c] = d.bodies[b].verts[3 * (w - off) + c];
            return;
          }
          off += d.bodies[b].nv;
        }
      }
    };
    C.tri0 = Ntr;
    for (const auto& t : tris)
      for (int k = 0; k < 3; ++k) h_trv.push_back(t[k]);
    C.tri1 = Ntr + (int)tris.size();
    H.tri0 = C.tri0;
    H.tri1 = C.tri1;
    std::vector<std::pair<int, int>> edges;
    for (const auto& t : tris)
      for (int k = 0; k < 3; ++k) {
        int a = t[k], b = t[(k + 1) % 3];
        if (a > b) std::swap(a, b);
        edges.emplace_back(a, b);
      }
    std::sort(edges.begin(), edges.end());
    edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
    C.edge0 = Ned;
    for (const auto& e : edges) {
      h_edv.push_back(e.first);
      h_edv.push_back(e.second);
      double pa[3], pb[3];
      rest_pos(e.first, pa);
      rest_pos(e.second, pb);
      h_elen2.push_back((pb[0] - pa[0]) * (pb[0] - pa[0]) + (pb[1] - pa[1]) * (pb[1] - pa[1]) +
                        (pb[2] - pa[2]) * (pb[2] - pa[2]));
    }
    C.edge1 = Ned + (int)edges.size();
    H.edge0 = C.edge0;
    H.edge1 = C.edge1;
    // queries: contact vertices (point-triangle) then edges (edge-edge), scene by scene
    C.q0 = Nq;
    for (int k = 0; k < ncv; ++k) {
      h_qkind.push_back(0);
      h_qidx.push_back(cv0 + k);
      h_qscene.push_back(s);
    }
    for (size_t k = 0; k < edges.size(); ++k) {
      h_qkind.push_back(1);
      h_qidx.push_back(Ned + (int)k);
      h_qscene.push_back(s);
    }
    C.q1 = Nq + ncv + (int)edges.size();
    // broad-phase grid: cell edge = mean edge extent + 2 dhat, origin below the scene's
    // bounding box
    double ext = 0.0;
    int next = 0;
    for (const auto& e : edges) {
      double pa[3], pb[3];
      rest_pos(e.first, pa);
      rest_pos(e.second, pb);
      ext += std::max(std::fabs(pa[0] - pb[0]), std::max(std::fabs(pa[1] - pb[1]), std::fabs(pa[2] - pb[2])));
      ++next;
    }
    C.cell = (next ? ext / next : 1e-3) + 2.0 * P.dhat;
    for (int c = 0; c < 3; ++c) C.org[c] = (std::isfinite(lo[c]) ? lo[c] : 0.0) - 2.0 * C.cell;
    double L = 0.0;
    for (int c = 0; c < 3; ++c)
      if (std::isfinite(lo[c])) L += (hi[c] - lo[c]) * (hi[c] - lo[c]);
    L = std::sqrt(L);
    C.stop = P.newton_tol * P.h * L;
    H.stop = C.stop;
    // block tables
    tn_sblk_h.push_back((int)tn_sc_h.size());
    for (int b0 = node0; b0 < node0 + nn; b0 += kNodeChunk) {
      tn_sc_h.push_back(s);
      tn_b0_h.push_back(b0);
      tn_b1_h.push_back(std::min(b0 + kNodeChunk, node0 + nn));
    }
    ts_sblk_h.push_back((int)ts_sc_h.size());
    for (int b0 = node0; b0 < node0 + nn; b0 += kRowChunk) {
      ts_sc_h.push_back(s);
      ts_b0_h.push_back(b0);
      ts_b1_h.push_back(std::min(b0 + kRowChunk, node0 + nn));
    }
    tt_sblk_h.push_back((int)tt_sc_h.size());
    for (int b0 = tet0; b0 < tet0 + nt; b0 += kTetChunk) {
      tt_sc_h.push_back(s);
      tt_b0_h.push_back(b0);
      tt_b1_h.push_back(std::min(b0 + kTetChunk, tet0 + nt));
    }
    Nn += nn;
    Nt += nt;
    Nb += nb;
    Ncv += ncv;
    Ntr += (int)tris.size();
    Ned += (int)edges.size();
    Nq = C.q1;
  }
  tn_sblk_h.push_back((int)tn_sc_h.size());
  tn_sblk_host = tn_sblk_h;
  tt_sblk_h.push_back((int)tt_sc_h.size());
  ts_sblk_h.push_back((int)ts_sc_h.size());
  nnz = (int)h_col.size();
  h_nscene.resize(Nn);
  // Size of the static (FEM) part of one sparse product: blocks of free rows, free nodes.
  spmv_static_blocks.assign(S, 0.0);
  spmv_free_nodes.assign(S, 0.0);
  for (int n = 0; n < Nn; ++n) {
    if (!h_nfree[n]) continue;
    spmv_free_nodes[h_nscene[n]] += 1.0;
    spmv_static_blocks[h_nscene[n]] += h_rowptr[n + 1] - h_rowptr[n];
  }
  // SoA tet arrays
  std::vector<int> h_tv(4 * (size_t)Nt);
  std::vector<double> h_Dminv(9 * (size_t)Nt);
  for (int t = 0; t < Nt; ++t) {
    for (int a = 0; a < 4; ++a) h_tv[(size_t)a * Nt + t] = h_tv_aos[4 * (size_t)t + a];
    for (int k = 0; k < 9; ++k) h_Dminv[(size_t)k * Nt + t] = h_Dminv_aos[9 * (size_t)t + k];
  }
  // ---- upload (everything above is host-side validation and setup)
  if (validate_only) return;
  // ---- coarse level of the preconditioner (rest state, formed once)
  std::vector<int> cg_blk_agg_h(tn_sc_h.size(), -1), cg_agg_b0_h, cg_agg_b1_h, cg_sc_a0_h(S, 0),
      cg_sc_m_h(S, 0);
  std::vector<long long> cg_sc_off_h(S, 0);
  std::vector<double> cg_d_h(3 * (size_t)Nn, 0.0), cg_ainv_h;
  for (int s = 0; s < S; ++s) {
    const HostScene& H = hs[s];
    const SceneConst& C = hsc[s];
    CoarseScene cs;
    cs.node0 = H.node0;
    cs.nv = H.nv;
    cs.nfree = h_nfree.data();
    cs.X = h_x.data();
    cs.mass = h_mass.data();
    cs.tet0 = C.tet0;
    cs.tet1 = C.tet1;
    cs.tv = h_tv_aos.data();
    cs.Dminv = h_Dminv_aos.data();
    cs.vol = h_tvol.data();
    cs.h = C.h;
    cs.mu = C.mu;
    cs.lam = C.lam;
    cs.tn_b0 = tn_b0_h.data();
    cs.bfirst = tn_sblk_h[s];
    cs.bend = tn_sblk_h[s + 1];
    cs.block = kNodeChunk;
    cs.max_agg = kCoarseMaxAgg;
    cg_sc_a0_h[s] = (int)cg_agg_b0_h.size();
    cg_sc_off_h[s] = (long long)cg_ainv_h.size();
    cg_sc_m_h[s] = build_coarse(cs, cg_blk_agg_h, cg_agg_b0_h, cg_agg_b1_h, cg_d_h, cg_ainv_h);
  }
  cg_on = cg_agg_b0_h.empty() ? 0 : 1;
  cg_mmax = 0;
  for (int m2 : cg_sc_m_h) cg_mmax = std::max(cg_mmax, m2);
  // TS blocks (16 rows) of each aggregate: both tables start at the scene's first node and
  // 64 is a multiple of 16, so the rows of a TN block are the TS blocks 4j .. 4j + 3
  static_assert(kNodeChunk % kRowChunk == 0, "TN blocks must hold whole TS blocks");
  constexpr int kTsPerTn = kNodeChunk / kRowChunk;
  // Per scene: the TS blocks of its j-th aggregate are [ts0 + j tsn, min(ts0 + (j + 1) tsn, tsend)).
  std::vector<int> cg_sc_ts0_h(S, 0), cg_sc_tsn_h(S, 0), cg_sc_tsend_h(S, 0);
  for (int sc = 0; sc < S; ++sc) {
    const int na = cg_sc_m_h[sc] / 6;
    if (na == 0) continue;
    const int a0 = cg_sc_a0_h[sc];
    const int grp = cg_agg_b1_h[a0] - cg_agg_b0_h[a0];
    cg_sc_ts0_h[sc] = ts_sblk_h[sc] + kTsPerTn * (cg_agg_b0_h[a0] - tn_sblk_h[sc]);
    cg_sc_tsn_h[sc] = kTsPerTn * grp;
    cg_sc_tsend_h[sc] = std::min(ts_sblk_h[sc] + kTsPerTn * (cg_agg_b1_h[a0 + na - 1] - tn_sblk_h[sc]),
                                 ts_sblk_h[sc + 1]);
    for (int j = 0; j < na; ++j) {
      const int a = a0 + j;
      const int t0 = cg_sc_ts0_h[sc] + cg_sc_tsn_h[sc] * j;
      const int t1 = std::min(t0 + cg_sc_tsn_h[sc], cg_sc_tsend_h[sc]);
      if (t0 >= t1 || t0 < ts_sblk_h[sc] || t1 > ts_sblk_h[sc + 1])
        throw ApiError(TACCEL_ERR_HIP, "internal: empty or foreign row-block range of an aggregate");
      for (int t = t0; t < t1; ++t)
        if (ts_sc_h[t] != sc || ts_b0_h[t] < tn_b0_h[cg_agg_b0_h[a]] || ts_b1_h[t] > tn_b1_h[cg_agg_b1_h[a] - 1])
          throw ApiError(TACCEL_ERR_HIP, "internal: row blocks do not nest in node blocks");
      // every row of the aggregate's node blocks is in one of its row blocks
      if (ts_b0_h[t0] != tn_b0_h[cg_agg_b0_h[a]] || ts_b1_h[t1 - 1] != tn_b1_h[cg_agg_b1_h[a] - 1])
        throw ApiError(TACCEL_ERR_HIP, "internal: row blocks do not cover an aggregate");
    }
  }
  if (!mem.stream) {
    // a stream of our own (default priority): the PCG chunks are captured into a graph,
    // which the null stream does not allow
    HIPCHECK(hipStreamCreateWithFlags(&mem.stream, hipStreamNonBlocking));
    mem.own_stream = true;
  }
  // two more streams (default priority) and the events that fork work onto them and join it back
  HIPCHECK(hipStreamCreateWithFlags(&mem.side, hipStreamNonBlocking));
  HIPCHECK(hipStreamCreateWithFlags(&mem.side2, hipStreamNonBlocking));
  HIPCHECK(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
  HIPCHECK(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
  HIPCHECK(hipEventCreateWithFlags(&ev_join2, hipEventDisableTiming));
  device_touched = true;
  Mem* m = &mem;
  d_sc.upload(m, hsc);
  x.upload(m, h_x);
  xrest.upload(m, h_x);
  xn.ensure(m, 3 * (size_t)Nn);
  xhat.ensure(m, 3 * (size_t)Nn);
  v.upload(m, std::vector<double>(3 * (size_t)Nn, 0.0));
  mass.upload(m, h_mass);
  nfree.upload(m, h_nfree);
  nscene.upload(m, h_nscene);
  nbody.upload(m, h_nbody);
  ntype.upload(m, h_ntype);
  tv.upload(m, h_tv);
  tscene.upload(m, h_tscene);
  Dminv.upload(m, h_Dminv);
  tvol.upload(m, h_tvol);
  rowptr.upload(m, h_rowptr);
  col.upload(m, h_col);
  diag.upload(m, h_diag);
  vptr.upload(m, h_vptr);
  vlist.upload(m, h_vlist);
  val.ensure(m, 9 * (size_t)nnz);
  bnode.upload(m, h_bnode);
  bscene.upload(m, h_bscene);
  bpres.upload(m, h_bpres);
  bsnap.upload(m, std::vector<int>(Nb, 0));
  bcv0.upload(m, h_bcv0);
  bcv1.upload(m, h_bcv1);
  bmass.upload(m, h_bmass);
  bvol.upload(m, h_bvol);
  bstar.upload(m, std::vector<double>(12 * (size_t)Nb, 0.0));
  blam.upload(m, std::vector<double>(12 * (size_t)Nb, 0.0));
  bkap.upload(m, std::vector<double>(Nb, 1e6));
  bgrad.ensure(m, 12 * (size_t)Nb);
  bhess.ensure(m, 144 * (size_t)Nb);
  bpinv.ensure(m, 144 * (size_t)Nb);
  cvn.upload(m, h_cvn);
  cvb.upload(m, h_cvb);
  cvx.upload(m, h_cvx);
  cvfix.upload(m, h_cvfix);
  cvscene.upload(m, h_cvscene);
  cvworld.upload(m, h_cvworld);
  cpos.ensure(m, 3 * (size_t)Ncv);
  cdisp.ensure(m, 3 * (size_t)Ncv);
  cend.ensure(m, 3 * (size_t)Ncv);
  trv.upload(m, h_trv);
  edv.upload(m, h_edv);
  elen2.upload(m, h_elen2);
  qkind.upload(m, h_qkind);
  qidx.upload(m, h_qidx);
  qscene.upload(m, h_qscene);
  act.upload(m, std::vector<int>(S, 0));
  pdone.upload(m, std::vector<int>(S, 1));
  exact.upload(m, std::vector<int>(S, 0));
  indef.upload(m, std::vector<int>(S, 0));
  tn_sc.upload(m, tn_sc_h);
  tn_b0.upload(m, tn_b0_h);
  tn_b1.upload(m, tn_b1_h);
  tn_sblk.upload(m, tn_sblk_h);
  tt_sc.upload(m, tt_sc_h);
  tt_b0.upload(m, tt_b0_h);
  tt_b1.upload(m, tt_b1_h);
  tt_sblk.upload(m, tt_sblk_h);
  TN.nblk = (int)tn_sc_h.size();
  TN.sc = tn_sc.p; TN.b0 = tn_b0.p; TN.b1 = tn_b1.p; TN.sblk = tn_sblk.p;
  TT.nblk = (int)tt_sc_h.size();
  TT.sc = tt_sc.p; TT.b0 = tt_b0.p; TT.b1 = tt_b1.p; TT.sblk = tt_sblk.p;
  ts_sc.upload(m, ts_sc_h);
  ts_b0.upload(m, ts_b0_h);
  ts_b1.upload(m, ts_b1_h);
  ts_sblk.upload(m, ts_sblk_h);
  TS.nblk = (int)ts_sc_h.size();
  TS.sc = ts_sc.p; TS.b0 = ts_b0.p; TS.b1 = ts_b1.p; TS.sblk = ts_sblk.p;
  // PCG / line-search / misc
  for (DBuf<double>* b : {&g, &r, &z, &p, &p1, &q, &dx}) b->ensure(m, 3 * (size_t)Nn);
  pinv.ensure(m, 9 * (size_t)Nn);
  for (DBuf<double>* b : {&P_rz0, &P_rz1, &P_gg}) b->ensure(m, std::max(TN.nblk, 1));
  P_pq.ensure(m, std::max(TS.nblk, 1));
  cg_blk_agg.upload(m, cg_blk_agg_h);
  cg_agg_b0.upload(m, cg_agg_b0_h.empty() ? std::vector<int>(1, 0) : cg_agg_b0_h);
  cg_agg_b1.upload(m, cg_agg_b1_h.empty() ? std::vector<int>(1, 0) : cg_agg_b1_h);
  cg_sc_a0.upload(m, cg_sc_a0_h);
  cg_sc_m.upload(m, cg_sc_m_h);
  cg_sc_off.upload(m, cg_sc_off_h);
  cg_rc.ensure(m, 6 * (size_t)std::max(TN.nblk, 1));
  P_qc.ensure(m, 6 * (size_t)std::max(TS.nblk, 1));
  cg_rca0.ensure(m, 6 * (size_t)std::max<size_t>(cg_agg_b0_h.size(), 1));
  cg_rca1.ensure(m, 6 * (size_t)std::max<size_t>(cg_agg_b0_h.size(), 1));
  cg_sc_ts0.upload(m, cg_sc_ts0_h);
  cg_sc_tsn.upload(m, cg_sc_tsn_h);
  cg_sc_tsend.upload(m, cg_sc_tsend_h);
  // FP32 staging copies stay alive until the stream synchronisation below
  const std::vector<float> af(cg_ainv_h.begin(), cg_ainv_h.end());
  cg_ainv.ensure(m, af.size() / 2 + 1);
  h2d(reinterpret_cast<float*>(cg_ainv.p), af.data(), af.size());
  // (d, w) per node for the restriction inside the sparse product: w = 1 where the coarse
  // offset is defined (free soft nodes of an aggregate)
  std::vector<double> dw_h(4 * (size_t)Nn, 0.0);
  for (int s2 = 0; s2 < S; ++s2) {
    if (cg_sc_m_h[s2] == 0) continue;
    const HostScene& H = hs[s2];
    for (int n = H.node0; n < H.node0 + H.nv; ++n) {
      if (!h_nfree[n] || cg_blk_agg_h[tn_sblk_h[s2] + (n - H.node0) / kNodeChunk] < 0) continue;
      for (int c = 0; c < 3; ++c) dw_h[4 * (size_t)n + c] = cg_d_h[3 * (size_t)n + c];
      dw_h[4 * (size_t)n + 3] = 1.0;
    }
  }
  std::vector<float> df, dwf;
  if (mixed) {
    df.assign(cg_d_h.begin(), cg_d_h.end());
    cg_d.ensure(m, df.size() / 2 + 1);
    h2d(reinterpret_cast<float*>(cg_d.p), df.data(), df.size());
    dwf.assign(dw_h.begin(), dw_h.end());
    cg_dw.ensure(m, dwf.size() / 2 + 1);
    h2d(reinterpret_cast<float*>(cg_dw.p), dwf.data(), dwf.size());
  } else {
    cg_d.upload(m, cg_d_h);
    cg_dw.upload(m, dw_h);
  }
  if (refine) {
    // the FP32 passes read FP32 coarse offsets; the system and its preconditioner are
    // converted from FP64 for every Newton direction
    cg_d32.upload(m, std::vector<float>(cg_d_h.begin(), cg_d_h.end()));
    cg_dw32.upload(m, std::vector<float>(dw_h.begin(), dw_h.end()));
    val32.ensure(m, 9 * (size_t)std::max(nnz, 1));
    pinv32.ensure(m, 9 * (size_t)std::max(Nn, 1));
    bpinv32.ensure(m, 144 * (size_t)std::max(Nb, 1));
    for (DBuf<double>* b : {&dxc, &gres}) b->ensure(m, 3 * (size_t)std::max(Nn, 1));
    rpart.ensure(m, 2 * (size_t)std::max(TN.nblk, 1));
  }
  sync();
  iters.ensure(m, S);
  fg_prev.ensure(m, 2 * (size_t)S);
  bad.ensure(m, S);
  infeasible.ensure(m, S);
  scnt.ensure(m, S + 1);
  cand_off.ensure(m, S + 1);
  okflag.ensure(m, S);
  failflag.ensure(m, S);
  action.ensure(m, std::max(Nb, 1));
  snapcand.ensure(m, std::max(Nb, 1));
  u64s.ensure(m, 2 * (size_t)S + Nb + 1);
  abase.ensure(m, S);
  alpha.ensure(m, S);
  dE.ensure(m, kTrials * (size_t)S);
  part_nodes.ensure(m, kTrials * (size_t)std::max(TN.nblk, 1));
  part_tets.ensure(m, kTrials * (size_t)std::max(TT.nblk, 1));
  e_bodies.ensure(m, (kTrials + 1) * (size_t)std::max(Nb, 1));
  scalars.ensure(m, 16);
  bp_ovf.ensure(m, std::max(S, 1));
  rowcnt.ensure(m, Nn + 1);
  drowptr.ensure(m, Nn + 1);
  bp.ntarget = Ntr + Ned;
  bp_tbox.ensure(m, 6 * (size_t)std::max(bp.ntarget, 1));
  bp_tcell.ensure(m, 6 * (size_t)std::max(bp.ntarget, 1));
  bp_tncell.ensure(m, std::max(bp.ntarget, 1));
  bp_toff.ensure(m, std::max(bp.ntarget, 1));
  bp_qcount.ensure(m, std::max(Nq, 1));
  bp_qoff.ensure(m, std::max(Nq, 1));
  HIPCHECK(hipHostMalloc((void**)&h_pin, kStageBytes, hipHostMallocDefault));
  h_pin_bytes = kStageBytes;
  h_pin_used = 0;
  // The initial state must have every admissible pair at positive distance (the barrier is
  // infinite at contact); tets were checked on the host.
  {
    const View V = view();
    launch_cpos(V, mem.stream);
    const int nc = broad_phase(cpos.p, nullptr, 1, cq, ct);
    zero(bad.p, sizeof(int) * S);
    launch_touching(V, nc, cq.p, ct.p, bad.p, mem.stream);
    std::vector<int> hb(S);
    d2h(hb.data(), bad.p, S);
    sync();
    for (int k = 0; k < S; ++k)
      if (hb[k]) throw ApiError(TACCEL_INFEASIBLE, "scene " + std::to_string(k) +
                                                       ": a contact pair is at zero distance");
  }
  sync();
}

// Candidates of the active scenes (or all scenes) for boxes over P0 (and P1).  Returns the
// count; oq/ot receive (query, target) in canonical (scene, kind, i, j) order.
int Batch::Impl::broad_phase(const double* P0, const double* P1, int all, DBuf<int>& oq,
                             DBuf<int>& ot, std::vector<int>* ovf) {
  const View V = view();
  hipStream_t s = stream();
  bp.tbox = bp_tbox.p;
  bp.tcell = bp_tcell.p;
  bp.tncell = bp_tncell.p;
  bp.toff = bp_toff.p;
  bp.qcount = bp_qcount.p;
  bp.qoff = bp_qoff.p;
  bp.overflow = bp_ovf.p;
  zero(bp.overflow, sizeof(int) * S);
  std::vector<int> flags(S);
  auto check = [&]() {
    bool any = false;
    for (int k = 0; k < S; ++k) any = any || flags[k];
    if (!any) return;
    if (!ovf)
      throw ApiError(TACCEL_NAN, "broad phase: a primitive box spans too many cells "
                                 "(positions exploded or non-finite)");
    for (int k = 0; k < S; ++k) (*ovf)[k] = (*ovf)[k] || flags[k];
  };
  if (ovf) ovf->assign(S, 0);
  launch_bp_targets(V, P0, P1, bp, all, s);
  scan_async(bp.tncell, bp.toff, bp.ntarget, scalars.p);
  int nentries = 0;
  d2h(&nentries, scalars.p, 1);
  d2h(flags.data(), bp.overflow, S);
  sync();
  check();  // boxes that overflowed were collapsed to one cell: the counts below are bounded
  long long table = 1024;
  while (table < 2 * (long long)nentries) table <<= 1;
  bp_bcount.ensure(&mem, table);
  bp_bstart.ensure(&mem, table);
  bp_bfill.ensure(&mem, table);
  bp_entries.ensure(&mem, std::max(nentries, 1));
  bp.table_mask = (int)(table - 1);
  bp.bcount = bp_bcount.p;
  bp.bstart = bp_bstart.p;
  bp.bfill = bp_bfill.p;
  bp.entries = bp_entries.p;
  zero(bp.bcount, sizeof(int) * table);
  zero(bp.bfill, sizeof(int) * table);
  launch_bp_count(V, bp, s);
  scan_async(bp.bcount, bp.bstart, (int)table, scalars.p + 2);
  launch_bp_fill(V, bp, s);
  launch_bp_query(V, P0, P1, bp, all, 0, nullptr, nullptr, nullptr, s);
  scan_async(bp.qcount, bp.qoff, Nq, scalars.p);
  int ncand = 0;
  d2h(&ncand, scalars.p, 1);
  d2h(flags.data(), bp.overflow, S);
  sync();
  check();
  oq.ensure(&mem, std::max(ncand, 1));
  ot.ensure(&mem, std::max(ncand, 1));
  bp_tmp.ensure(&mem, std::max(ncand, 1));
  launch_bp_query(V, P0, P1, bp, all, 1, oq.p, ot.p, bp_tmp.p, s);
  return ncand;
}

template <class T>
PcgBufsT<T> Batch::Impl::pcg_bufs() {
  PcgBufsT<T> B;
  B.g = g.p;
  B.r = reinterpret_cast<T*>(r.p);
  B.z = reinterpret_cast<T*>(z.p);
  B.p0 = reinterpret_cast<T*>(p.p);
  B.p1 = reinterpret_cast<T*>(p1.p);
  B.q = reinterpret_cast<T*>(q.p);
  B.dx = dx.p;
  B.pinv = reinterpret_cast<const T*>(pinv.p);
  B.drowptr = drowptr.p;
  B.dcol = dcol.p;
  B.dval = reinterpret_cast<const T*>(dval.p);
  B.P_pq = reinterpret_cast<T*>(P_pq.p);
  B.P_rz0 = reinterpret_cast<T*>(P_rz0.p);
  B.P_rz1 = reinterpret_cast<T*>(P_rz1.p);
  B.P_gg = reinterpret_cast<T*>(P_gg.p);
  B.keep_gg = 0;
  B.ggprev = fg_prev.p;
  B.etaprev = fg_prev.p + S;
  B.iters = iters.p;
  B.indef = indef.p;
  B.cg_on = cg_on;
  B.cg_mmax = cg_on ? cg_mmax : 0;
  B.cg_blk_agg = cg_blk_agg.p;
  B.cg_agg_b0 = cg_agg_b0.p;
  B.cg_agg_b1 = cg_agg_b1.p;
  B.cg_sc_a0 = cg_sc_a0.p;
  B.cg_sc_m = cg_sc_m.p;
  B.cg_sc_off = cg_sc_off.p;
  B.cg_d = reinterpret_cast<const T*>(cg_d.p);
  B.cg_dw = reinterpret_cast<const T*>(cg_dw.p);
  B.cg_ainv = reinterpret_cast<const float*>(cg_ainv.p);
  B.cg_rc = reinterpret_cast<T*>(cg_rc.p);
  B.cg_sc_ts0 = cg_sc_ts0.p;
  B.cg_sc_tsn = cg_sc_tsn.p;
  B.cg_sc_tsend = cg_sc_tsend.p;
  B.P_qc = reinterpret_cast<T*>(P_qc.p);
  B.cg_rca0 = reinterpret_cast<T*>(cg_rca0.p);
  B.cg_rca1 = reinterpret_cast<T*>(cg_rca1.p);
  int max_pcg = 0;
  for (const auto& H : hs) max_pcg = std::max(max_pcg, H.max_pcg);
  B.max_iters = max_pcg;
  return B;
}

template <class T>
void Batch::Impl::run_pcg(const View& V, const PcgBufsT<T>& B, const int* nseg_d) {
  hipStream_t s = stream();
  Profiler& prof = profiler();
  double launch_bytes = 0.0;
  if (prof.on) {
    const int nseg = read_int(nseg_d);  // dynamic blocks of this matrix
    std::vector<int> ha(S);
    d2h(ha.data(), act.p, S);
    sync();
    // static part: per free row its blocks (9 values + 4 B column), 4 B row pointer, 4 B flag,
    // x read and y written once
    const double w0 = sizeof(T);
    for (int k = 0; k < S; ++k)
      if (ha[k]) launch_bytes += (9 * w0 + 4.0) * spmv_static_blocks[k] + (8.0 + 6 * w0) * spmv_free_nodes[k];
    // dynamic (contact and body) blocks: values + 4 B column each, 4 B row pointer per
    // node; the direction update adds z and p_{k-1} read and p_k written per free node
    const double w = sizeof(T);
    launch_bytes += (9 * w + 4.0) * nseg + 4.0 * Nn;
    for (int k = 0; k < S; ++k)
      if (ha[k]) launch_bytes += 9.0 * w * spmv_free_nodes[k];
    // with the coarse level: the rest offset and weight of every row (4 values) read and the
    // restriction of q (6 values per 16-row block) written; p.q partials (1 value per block)
    for (int k = 0; k < S; ++k)
      if (ha[k]) {
        const int nrow = hs[k].node1 - hs[k].node0;
        const double rows = nrow, blocks = (nrow + kRowChunk - 1) / kRowChunk;
        launch_bytes += w * blocks + (B.cg_on ? 4.0 * w * rows + 6.0 * w * blocks : 0.0);
      }
  }
  if (prof.on)
    while (ev_pool.size() < 2 * (size_t)kPcgChunk) {
      hipEvent_t e;
      HIPCHECK(hipEventCreate(&e));
      ev_pool.push_back(e);
    }
  std::vector<int> hd(S);
  if (prof.on) {
    // Live sample of the sparse product on this Newton iteration's matrix: kSample launches
    // back to back between one pair of events, right after the PCG initialisation.  The
    // launches only write p_1, q and the p.q partials, which iteration 0 recomputes.
    constexpr int kSample = 16;
    HIPCHECK(hipEventRecord(ev_pool[0], s));
    for (int k = 0; k < kSample; ++k) launch_pcg_spmv(V, TN, TS, B, 0, s);
    HIPCHECK(hipEventRecord(ev_pool[1], s));
    HIPCHECK(hipEventSynchronize(ev_pool[1]));
    float ms = 0.f;
    HIPCHECK(hipEventElapsedTime(&ms, ev_pool[0], ev_pool[1]));
    prof.spmv_ms += ms;
    prof.spmv_launches += kSample;
    prof.spmv_bytes += kSample * launch_bytes;
  }
  const std::vector<const void*> key = {B.dval, B.dcol, B.drowptr, B.pinv, B.dx, V.bpinv, V.val};
  if (!pcg_exec || key != pcg_key) {
    // (re)capture the chunk; when only buffer addresses changed, the existing executable
    // graph is updated in place rather than rebuilt
    HIPCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < kPcgChunk; ++k) {
      launch_pcg_spmv(V, TN, TS, B, k & 1, s);
      launch_pcg_update(V, TN, TS, B, k & 1, s);
    }
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &graph);  // always ends the capture
    if (ec != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      HIPCHECK(ec);
    }
    bool updated = false;
    if (pcg_exec) {
      hipGraphNode_t err_node = nullptr;
      hipGraphExecUpdateResult res = hipGraphExecUpdateError;
      updated = hipGraphExecUpdate(pcg_exec, graph, &err_node, &res) == hipSuccess &&
                res == hipGraphExecUpdateSuccess;
      if (!updated) {
        (void)hipGetLastError();
        HIPCHECK(hipGraphExecDestroy(pcg_exec));
        pcg_exec = nullptr;
      }
    }
    if (!updated) {
      for (hipGraph_t g0 : pcg_graphs) HIPCHECK(hipGraphDestroy(g0));
      pcg_graphs.clear();
    }
    pcg_graphs.push_back(graph);  // owned from here on, also if instantiation fails
    if (!updated) HIPCHECK(hipGraphInstantiate(&pcg_exec, graph, nullptr, nullptr, 0));
    pcg_key = key;
  }
  // chunks launched before the first convergence check: about 3/4 of the previous solve's
  // iteration count (chunks after convergence return at once)
  const int nfirst = std::max(1, std::min(8, (3 * pcg_last_max / 4) / kPcgChunk));
  if (prof.on) HIPCHECK(hipEventRecord(ev_pool[2], s));
  for (int it = 0; it < B.max_iters; it += kPcgChunk) {
    if (it == 0)
      for (int c = 1; c < nfirst && (c + 1) * kPcgChunk <= B.max_iters; ++c, it += kPcgChunk)
        HIPCHECK(hipGraphLaunch(pcg_exec, s));
    HIPCHECK(hipGraphLaunch(pcg_exec, s));
    d2h(hd.data(), pdone.p, S);
    sync();
    bool all = true;
    for (int k = 0; k < S; ++k) all = all && hd[k];
    if (all) break;
  }
  if (prof.on) {
    HIPCHECK(hipEventRecord(ev_pool[3], s));
    HIPCHECK(hipEventSynchronize(ev_pool[3]));
    float ms = 0.f;
    HIPCHECK(hipEventElapsedTime(&ms, ev_pool[2], ev_pool[3]));
    std::vector<int> it(S);
    d2h(it.data(), iters.p, S);
    sync();
    int mx = 0;
    for (int v : it) mx = std::max(mx, v);
    prof.pcg_ms += ms;
    prof.pcg_iters += mx;
  }
}

// FP32 PCG with FP64 refinement (TACCEL_FP64_REFINED) for the scenes of act_s (the device's
// act holds the same set; the directions of the other scenes are left as they are): the FP64
// blocks and block-Jacobi inverses are rounded to FP32 once; each pass runs the FP32 PCG on
// the current residual and adds its solution to dx in FP64; after a pass the FP64 residual
// gres = g + H dx is measured in the FP64 block-Jacobi norm, and a scene whose
// gres^T D^-1 gres exceeds eta^2 g^T D^-1 g (and whose pass met no direction of non-positive
// curvature) takes another pass, at most kRefinePasses in all.  The passes' stopping test keeps
// the first pass's reference, so every pass aims at eta relative to the Newton gradient.
// Returns the PCG iterations per scene, summed over the passes.
std::vector<int> Batch::Impl::solve_refined(const View& V, const int* nseg_d, const std::vector<int>& act_s) {
  hipStream_t s = stream();
  launch_to_f32(9 * (size_t)nnz, V.val, val32.p, s);
  launch_to_f32(9 * (size_t)std::max(nh_last, 0), dval.p, dval32.p, s);
  launch_to_f32(9 * (size_t)Nn, pinv.p, pinv32.p, s);
  launch_to_f32(144 * (size_t)Nb, bpinv.p, bpinv32.p, s);
  View V32 = V;
  V32.val = reinterpret_cast<double*>(val32.p);      // read as FP32 by the PCG kernels
  V32.bpinv = reinterpret_cast<double*>(bpinv32.p);  // the same
  PcgBufsT<float> B = pcg_bufs<float>();
  B.pinv = pinv32.p;
  B.dval = dval32.p;
  B.cg_d = cg_d32.p;
  B.cg_dw = cg_dw32.p;
  B.dx = dxc.p;
  std::vector<int> total(S, 0), pending = act_s, it_h(S), indef_h(S);
  std::vector<double> part;
  for (int pass = 0;; ++pass) {
    // pdone = !pending was set by the caller for the first pass
    zero(iters.p, sizeof(int) * S);
    zero(dxc.p, sizeof(double) * 3 * (size_t)Nn);  // scenes skipped by the pass add zero
    launch_pcg_init(V32, TN, B, s);
    launch_pcg_coarse(V32, TN, B, B.P_rz0, s);
    run_pcg(V32, B, nseg_d);
    launch_refine_apply(V, dxc.p, dx.p, pass == 0, s);
    d2h(it_h.data(), iters.p, S);
    d2h(indef_h.data(), indef.p, S);
    sync();
    Profiler& prof = profiler();
    for (int k = 0; k < S; ++k)
      if (pending[k]) {
        total[k] += it_h[k];
        if (prof.on) {
          prof.refine_passes += 1;
          prof.refine_dirs += pass == 0;
        }
      }
    if (pass + 1 == kRefinePasses) break;
    // FP64 residual of the scenes that took this pass
    std::vector<int> hd(S);
    for (int k = 0; k < S; ++k) hd[k] = !pending[k];
    h2d(pdone.p, hd.data(), S);
    launch_refine_resid(V, TS, drowptr.p, dcol.p, dval.p, g.p, dx.p, gres.p, s);
    launch_refine_norm(V, TN, pinv.p, g.p, gres.p, rpart.p, s);
    part.resize(2 * (size_t)std::max(TN.nblk, 1));
    d2h(part.data(), rpart.p, part.size());
    if (pass == 0) gg_readback();  // the first pass's reference: the tolerance it used
    sync();
    bool any = false;
    for (int k = 0; k < S; ++k) {
      if (!pending[k]) continue;
      double rr = 0.0, gg = 0.0;  // block order: the same sum on every call
      for (int b = tn_sblk_host[k]; b < tn_sblk_host[k + 1]; ++b) {
        rr += part[2 * (size_t)b];
        gg += part[2 * (size_t)b + 1];
      }
      const double eta = eta_used(k);
      pending[k] = !indef_h[k] && std::isfinite(rr) && rr > eta * eta * gg;
      any = any || pending[k];
    }
    if (!any) break;
    for (int k = 0; k < S; ++k) hd[k] = !pending[k];
    h2d(pdone.p, hd.data(), S);
    B.g = gres.p;
    B.keep_gg = 1;
  }
  return total;
}

// Friction pairs of the step (Taccel App. A.3): every pair closer than dhat at the
// start-of-step positions in a scene with friction, with its lagged closest-point weights,
// normal and mu * lambda, grouped by scene.
// Pairs of scene k closer than dhat at the current positions (broad and narrow phase on the
// device), as 5-int records in the caller's world vertex ids, sorted.
std::vector<int32_t> Batch::Impl::contacts(int k) {
  hipStream_t s = stream();
  View V = view();
  std::vector<int> on(S, 0);
  on[k] = 1;
  h2d(act.p, on.data(), S);
  launch_cpos(V, s);
  const int nc = broad_phase(cpos.p, nullptr, 0, cq, ct);
  cflag.ensure(&mem, std::max(nc, 1));
  cpos_idx.ensure(&mem, std::max(nc, 1));
  launch_narrow(V, nc, cq.p, ct.p, cflag.p, s);
  const int np = scan(cflag.p, cpos_idx.p, nc);
  DBuf<int> rec;
  rec.ensure(&mem, 5 * (size_t)std::max(np, 1));
  launch_contact_records(V, nc, cq.p, ct.p, cflag.p, cpos_idx.p, rec.p, s);
  std::vector<int32_t> out(5 * (size_t)np);
  d2h(out.data(), rec.p, out.size());
  sync();
  rec.free();
  cover_valid = false;
  std::vector<std::array<int32_t, 5>> r(np);
  for (int i = 0; i < np; ++i)
    for (int j = 0; j < 5; ++j) r[i][j] = out[5 * (size_t)i + j];
  std::sort(r.begin(), r.end());
  for (int i = 0; i < np; ++i)
    for (int j = 0; j < 5; ++j) out[5 * (size_t)i + j] = r[i][j];
  return out;
}

void Batch::Impl::build_friction(const int* mask) {
  hipStream_t s = stream();
  std::vector<int> on(S, 0);
  bool any = false;
  for (int k = 0; k < S; ++k) {
    on[k] = (!mask || mask[k]) && hsc[k].fmu > 0.0;
    any = any || on[k];
  }
  if (!any) return;
  h2d(act.p, on.data(), S);
  View V = view();
  launch_cpos(V, s);
  std::vector<int> overflow(S, 0);
  const int ncand = broad_phase(cpos.p, nullptr, 0, cq, ct, &overflow);
  cflag.ensure(&mem, std::max(ncand, 1));
  cpos_idx.ensure(&mem, std::max(ncand, 1));
  launch_narrow(V, ncand, cq.p, ct.p, cflag.p, s);
  const int n = scan(cflag.p, cpos_idx.p, ncand);
  pkind.ensure(&mem, std::max(n, 1));
  pv.ensure(&mem, 4 * (size_t)std::max(n, 1));
  pmeps.ensure(&mem, std::max(n, 1));
  pscene.ensure(&mem, std::max(n, 1));
  launch_compact_pairs(V, ncand, cq.p, ct.p, cflag.p, cpos_idx.p, pkind.p, pv.p, pmeps.p, pscene.p, s);
  fv.ensure(&mem, 4 * (size_t)std::max(n, 1));
  fw.ensure(&mem, 4 * (size_t)std::max(n, 1));
  fc0.ensure(&mem, 3 * (size_t)std::max(n, 1));
  fnrm.ensure(&mem, 3 * (size_t)std::max(n, 1));
  fmul.ensure(&mem, std::max(n, 1));
  fsoff.ensure(&mem, S + 1);
  nfric = n;
  launch_fric_build(V, n, pkind.p, pv.p, pmeps.p, fric_bufs(), s);
  // per-scene ranges (the candidates, hence the pairs, come grouped by scene)
  zero(scnt.p, sizeof(int) * (S + 1));
  launch_count_scene(n, pscene.p, scnt.p, s);
  std::vector<int> cnt(S);
  d2h(cnt.data(), scnt.p, S);
  sync();
  std::vector<int> off(S + 1, 0);
  for (int k = 0; k < S; ++k) off[k + 1] = off[k] + cnt[k];
  if (off[S] != n) throw ApiError(TACCEL_ERR_HIP, "internal: friction pair count mismatch");
  h2d(fsoff.p, off.data(), S + 1);
}

// Pairs closer than dhat at the current positions of the iterating scenes, compacted into the
// pair arrays (kind, vertices, mollifier threshold, scene) with per-scene counts; returns their
// number.  bp_bad flags scenes whose boxes overflowed the grid.
int Batch::Impl::prepare_pairs(std::vector<int>& bp_bad) {
  hipStream_t s = stream();
  View V = view();
  launch_cpos(V, s);
  // ---- active pairs at the current point: from the covering set of the previous
  // iteration when it is still valid, else from a static broad phase
  int ncand;
  const int* cqp;
  const int* ctp;
  if (cover_valid) {
    ncand = n_cover;
    cqp = sq.p;
    ctp = st.p;
  } else {
    ncand = broad_phase(cpos.p, nullptr, 0, cq, ct, &bp_bad);
    cqp = cq.p;
    ctp = ct.p;
  }
  cflag.ensure(&mem, std::max(ncand, 1));
  cpos_idx.ensure(&mem, std::max(ncand, 1));
  launch_narrow(V, ncand, cqp, ctp, cflag.p, s);
  const int np = scan(cflag.p, cpos_idx.p, ncand);
  // the step's friction pairs follow the barrier pairs in the pair arrays
  const int npf = np + nfric;
  pkind.ensure(&mem, std::max(np, 1));
  pv.ensure(&mem, 4 * (size_t)std::max(npf, 1));
  pmeps.ensure(&mem, std::max(np, 1));
  pscene.ensure(&mem, std::max(np, 1));
  pg.ensure(&mem, 12 * (size_t)std::max(npf, 1));
  ph.ensure(&mem, 144 * (size_t)std::max(npf, 1));
  launch_compact_pairs(V, ncand, cqp, ctp, cflag.p, cpos_idx.p, pkind.p, pv.p, pmeps.p, pscene.p, s);
  zero(scnt.p, sizeof(int) * (S + 1));
  launch_count_scene(np, pscene.p, scnt.p, s);
  return np;
}

// Gradient and Newton-system blocks of the iterating scenes at the current positions, for the
// np pairs prepared above and the step's friction pairs after them (npf in all): element
// derivatives, the static FEM blocks, and the contact and body blocks emitted, sorted by
// (row, col) and reduced into the dynamic block rows.  Returns the device count of dynamic
// blocks.
int* Batch::Impl::derivatives(int np, int npf) {
  hipStream_t s = stream();
  View V = view();
  // ---- element derivatives
  // Three independent chains, joined before the contact blocks are reduced: the contact
  // Hessians (one wavefront per pair: long and narrow) on the second stream, the FEM and
  // affine-body terms with the static assembly on the third, and the emission and sort of the
  // contact blocks here.
  HIPCHECK(hipEventRecord(ev_fork, s));
  HIPCHECK(hipStreamWaitEvent(mem.side, ev_fork, 0));
  HIPCHECK(hipStreamWaitEvent(mem.side2, ev_fork, 0));
  launch_barrier_hess(V, np, pkind.p, pv.p, pmeps.p, pg.p, ph.p, mem.side);
  HIPCHECK(hipEventRecord(ev_join, mem.side));
  launch_fem_rows(V, g.p, mixed, mem.side2);
  launch_body_hess(V, mem.side2);
  HIPCHECK(hipEventRecord(ev_join2, mem.side2));
  // ---- contact and body blocks: emit, sort by (row, col), reduce
  if (nfric > 0) launch_fric_derivs(V, fric_bufs(), np, pv.p, pg.p, ph.p, s);
  const int nitems = npf + Nb;
  hcnt.ensure(&mem, std::max(nitems, 1));
  gcnt.ensure(&mem, std::max(nitems, 1));
  hoff.ensure(&mem, std::max(nitems, 1));
  goff.ensure(&mem, std::max(nitems, 1));
  launch_contrib_count(V, npf, pv.p, hcnt.p, gcnt.p, s);
  scan_async(hcnt.p, hoff.p, nitems, scalars.p + 3);
  scan_async(gcnt.p, goff.p, nitems, scalars.p + 4);
  int hg[2];
  d2h(hg, scalars.p + 3, 2);
  sync();
  const int nh = hg[0], ng = hg[1];
  for (DBuf<uint64_t>* b : {&hkey, &hkey2}) b->ensure(&mem, std::max(nh, 1));
  for (DBuf<int>* b : {&hidx, &hidx2, &hsrc}) b->ensure(&mem, std::max(nh, 1));
  hcoef.ensure(&mem, std::max(nh, 1));
  for (DBuf<uint64_t>* b : {&gkey, &gkey2}) b->ensure(&mem, std::max(ng, 1));
  for (DBuf<int>* b : {&gidx, &gidx2, &gsrc}) b->ensure(&mem, std::max(ng, 1));
  gcoef.ensure(&mem, std::max(ng, 1));
  launch_contrib_emit(V, npf, pv.p, hoff.p, goff.p, hkey.p, hidx.p, hsrc.p, hcoef.p, gkey.p, gidx.p,
                      gsrc.p, gcoef.p, s);
  sort(hkey.p, hidx.p, hkey2.p, hidx2.p, nh, bits_for((uint64_t)Nn * (uint64_t)Nn));
  sort(gkey.p, gidx.p, gkey2.p, gidx2.p, ng, bits_for((uint64_t)Nn));
  const int nmax = std::max(nh, ng);
  sflag.ensure(&mem, std::max(nmax, 1));
  segid.ensure(&mem, std::max(nmax, 1));
  segstart.ensure(&mem, std::max(nmax, 1) + 1);
  // Hessian blocks.  The segment counts stay on the device (scalars 6 and 7): the records
  // bound them, so buffers and grids are sized by the record counts and the reductions read
  // the exact counts themselves.
  int* nseg_d = scalars.p + 6;
  int* ngseg_d = scalars.p + 7;
  launch_seg_flags(nh, hkey.p, sflag.p, s);
  scan_async(sflag.p, segid.p, nh, nseg_d);
  launch_seg_start(nh, sflag.p, segid.p, segstart.p, s);
  drow.ensure(&mem, std::max(nh, 1));
  dcol.ensure(&mem, std::max(nh, 1));
  dval.ensure(&mem, 9 * (size_t)std::max(nh, 1));
  if (refine) dval32.ensure(&mem, 9 * (size_t)std::max(nh, 1));
  nh_last = nh;
  zero(rowcnt.p, sizeof(int) * (Nn + 1));
  HIPCHECK(hipStreamWaitEvent(s, ev_join, 0));
  HIPCHECK(hipStreamWaitEvent(s, ev_join2, 0));
  launch_reduce_blocks(V, nh, nseg_d, hkey.p, hidx.p, segstart.p, hsrc.p, hcoef.p, ph.p, drow.p,
                       dcol.p, dval.p, rowcnt.p, mixed, s);
  scan_async(rowcnt.p, drowptr.p, Nn + 1, scalars.p + 5);
  // gradient entries
  launch_seg_flags(ng, gkey.p, sflag.p, s);
  scan_async(sflag.p, segid.p, ng, ngseg_d);
  launch_seg_start(ng, sflag.p, segid.p, segstart.p, s);
  launch_reduce_grad(V, ng, ngseg_d, gkey.p, gidx.p, segstart.p, gsrc.p, gcoef.p, pg.p, g.p, s);
  return nseg_d;
}

void Batch::Impl::newton_iteration(std::vector<int>& last, std::vector<int>& ls_fail,
                                   std::vector<int>& nan_, std::vector<int>& pcg_it,
                                   std::vector<int>& n_active, std::vector<int>& halvings) {
  hipStream_t s = stream();
  View V = view();
  Profiler& prof = profiler();
  auto t_mark = std::chrono::steady_clock::now();
  auto phase_end = [&](int ph) {  // profiling only: attribute the wall time since the last mark
    if (!prof.phases) return;
    sync();
    const auto now = std::chrono::steady_clock::now();
    prof.phase_ms[ph] += std::chrono::duration<double, std::milli>(now - t_mark).count();
    t_mark = now;
  };
  if (prof.phases) ++prof.phase_calls;
  std::vector<int> bp_bad(S, 0), bp_bad2(S, 0);  // scenes whose boxes overflowed the grid
  const int np = prepare_pairs(bp_bad);
  const int npf = np + nfric;
  phase_end(0);
  // Exact (unprojected) FEM and barrier Hessians for the scenes whose previous iteration of
  // this Newton loop took the full step with max vertex displacement <= 1e-2 dhat; the
  // projected ones otherwise, and again, in this same iteration, for a scene whose exact
  // system PCG finds not positive definite.
  std::vector<int> hbad(S, 0);
  for (int k = 0; k < S; ++k) {
    exact_h[k] = act_host[k] && prev_alpha[k] == 1.0 && prev_pmax[k] <= 1e-2 * hsc[k].dhat;
    pcg_it[k] = 0;
  }
  std::vector<int> attempt_act = act_host;
  // convergence measure of the Newton direction (max vertex displacement per scene), read
  // back with the solve's counters: one synchronisation for both
  unsigned long long* pmax = u64s.p;
  unsigned long long* amin = u64s.p + S;
  std::vector<unsigned long long> hp(S, 0ull), hp_att(S);
  std::vector<int> hcount(S);
  {
    std::vector<double> fg(2 * (size_t)S);
    for (int k = 0; k < S; ++k) {
      fg[k] = gg_prev_h[k];
      fg[S + k] = eta_prev_h[k];
    }
    h2d(fg_prev.p, fg.data(), fg.size());
  }
  for (int attempt = 0;; ++attempt) {
    h2d(exact.p, exact_h.data(), S);
    zero(indef.p, sizeof(int) * S);
    int* nseg_d = derivatives(np, npf);
    // ---- preconditioner and PCG
    zero(bad.p, sizeof(int) * S);
    launch_precond(V, drowptr.p, dcol.p, dval.p, pinv.p, bad.p, mixed, s);
    {
      // pdone = !act
      std::vector<int> ha(S);
      for (int k = 0; k < S; ++k) ha[k] = !attempt_act[k];
      h2d(pdone.p, ha.data(), S);
    }
    zero(iters.p, sizeof(int) * S);
    phase_end(1);
    std::vector<int> it_h(S), bad_h(S), indef_h(S);
    if (mixed) {
      const PcgBufsT<float> B = pcg_bufs<float>();
      launch_pcg_init(V, TN, B, s);
      launch_pcg_coarse(V, TN, B, B.P_rz0, s);
      run_pcg(V, B, nseg_d);
    } else if (refine) {
      it_h = solve_refined(V, nseg_d, attempt_act);
    } else {
      const PcgBufsT<double> B = pcg_bufs<double>();
      launch_pcg_init(V, TN, B, s);
      launch_pcg_coarse(V, TN, B, B.P_rz0, s);
      run_pcg(V, B, nseg_d);
    }
    phase_end(2);
    zero(pmax, sizeof(unsigned long long) * S);
    launch_pmax(V, dx.p, pmax, s);  // the scenes of this attempt (device act)
    if (!refine) d2h(it_h.data(), iters.p, S);
    d2h(bad_h.data(), bad.p, S);
    d2h(indef_h.data(), indef.p, S);
    d2h(hp_att.data(), pmax, S);
    if (attempt == 0) d2h(hcount.data(), scnt.p, S);
    gg_readback();
    sync();
    bool retry = false;
    for (int k = 0; k < S; ++k) {
      if (!attempt_act[k]) continue;
      hp[k] = hp_att[k];
      pcg_it[k] += it_h[k];
      hbad[k] = bad_h[k];
      attempt_act[k] = exact_h[k] && indef_h[k];
      if (attempt_act[k]) {
        exact_h[k] = 0;
        retry = true;
      }
    }
    if (!retry || attempt > 0) break;
    h2d(act.p, attempt_act.data(), S);
  }
  h2d(act.p, act_host.data(), S);
  // forcing-term state for the next iteration of each loop
  for (int k = 0; k < S; ++k)
    if (act_host[k] && hsc[k].forcing) {
      const double e = eta_used(k);
      gg_prev_h[k] = gg_scene(k);
      eta_prev_h[k] = e;
    }
  // ---- convergence check on the Newton direction (hp, read with the last solve)
  const std::vector<int>& hact = act_host;
  pcg_last_max = 0;
  for (int k = 0; k < S; ++k) {
    n_active[k] = hcount[k];
    if (hact[k]) pcg_last_max = std::max(pcg_last_max, pcg_it[k]);
  }
  for (int k = 0; k < S; ++k) {
    double pm;
    std::memcpy(&pm, &hp[k], sizeof(double));
    nan_[k] = hbad[k] || !std::isfinite(pm) || bp_bad[k];
    last[k] = pm <= hs[k].stop;
    if (act_host[k]) prev_pmax[k] = pm;
  }
  // a scene with a non-finite direction (or an exploded box) takes no further part in this
  // iteration: its sweep would cover the whole grid
  {
    bool any = false;
    std::vector<int> a2 = act_host;
    for (int k = 0; k < S; ++k)
      if (nan_[k] && a2[k]) {
        a2[k] = 0;
        any = true;
      }
    if (any) h2d(act.p, a2.data(), S);
  }
  phase_end(3);
  // ---- CCD over the swept candidates
  launch_cdisp(V, dx.p, s);
  launch_cend(V, cend.p, s);
  const int nsw = broad_phase(cpos.p, cend.p, 0, sq, st, &bp_bad2);
  for (int k = 0; k < S; ++k) nan_[k] = nan_[k] || bp_bad2[k];
  n_cover = nsw;
  cover_valid = true;
  {
    std::vector<unsigned long long> one(S);
    const double d1 = 1.0;
    unsigned long long b1;
    std::memcpy(&b1, &d1, sizeof(double));
    std::fill(one.begin(), one.end(), b1);
    h2d(amin, one.data(), S);
  }
  launch_ccd(V, nsw, sq.p, st.p, amin, s);
  std::vector<unsigned long long> ha(S);
  d2h(ha.data(), amin, S);
  launch_scene_offsets(V, nsw, sq.p, cand_off.p, s);
  std::vector<int> hoffs(S + 1);
  d2h(hoffs.data(), cand_off.p, S + 1);
  sync();
  std::vector<double> amax(S), alpha_h(S, 0.0);
  for (int k = 0; k < S; ++k) std::memcpy(&amax[k], &ha[k], sizeof(double));
  // blocks of at most kPairChunk swept candidates of one scene (line-search partial sums)
  {
    tp_sc_h.clear();
    tp_c0_h.clear();
    tp_c1_h.clear();
    tp_sblk_h.assign(1, 0);
    for (int k = 0; k < S; ++k) {
      for (int c0 = hoffs[k]; c0 < hoffs[k + 1]; c0 += kPairChunk) {
        tp_sc_h.push_back(k);
        tp_c0_h.push_back(c0);
        tp_c1_h.push_back(std::min(c0 + kPairChunk, hoffs[k + 1]));
      }
      tp_sblk_h.push_back((int)tp_sc_h.size());
    }
    // through the pinned staging area (no wait; large tables wait for their copy)
    for (const auto& pr : {std::make_pair(&tp_sc, &tp_sc_h), std::make_pair(&tp_b0, &tp_c0_h),
                     std::make_pair(&tp_b1, &tp_c1_h), std::make_pair(&tp_sblk, &tp_sblk_h)}) {
      pr.first->ensure(&mem, std::max<size_t>(pr.second->size(), 1));
      h2d(pr.first->p, pr.second->data(), pr.second->size());
    }
    TP.nblk = (int)tp_sc_h.size();
    TP.sc = tp_sc.p;
    TP.b0 = tp_b0.p;
    TP.b1 = tp_b1.p;
    TP.sblk = tp_sblk.p;
    part_pairs.ensure(&mem, kTrials * (size_t)std::max(TP.nblk, 1));
  }
  phase_end(4);
  // ---- line search (8 step sizes per launch)
  e_pairs.ensure(&mem, (kTrials + 1) * (size_t)std::max(nsw, 1));
  LsBufs L;
  L.p = dx.p;
  L.abase = abase.p;
  L.part_nodes = part_nodes.p;
  L.part_tets = part_tets.p;
  L.e_bodies = e_bodies.p;
  L.e_pairs = e_pairs.p;
  L.infeasible = infeasible.p;
  L.cand_off = cand_off.p;
  L.part_pairs = part_pairs.p;
  L.dE = dE.p;
  e_fric.ensure(&mem, (kTrials + 1) * (size_t)std::max(nfric, 1));
  L.F = fric_bufs();
  L.e_fric = e_fric.p;
  std::vector<int> pending(S, 0);
  std::vector<double> base(S);
  int npending = 0;
  for (int k = 0; k < S; ++k) {
    ls_fail[k] = 0;
    halvings[k] = 0;
    if (!hact[k] || nan_[k]) continue;
    if (last[k]) {
      alpha_h[k] = amax[k];
    } else {
      pending[k] = 1;
      ++npending;
    }
    base[k] = amax[k];
  }
  std::vector<double> hdE(kTrials * (size_t)S);
  std::vector<int> hinf(S);
  for (int round = 0; npending > 0; ++round) {
    h2d(abase.p, base.data(), S);
    zero(infeasible.p, sizeof(int) * S);
    launch_line_search(V, TN, TT, TP, nsw, sq.p, st.p, L, s);
    d2h(hdE.data(), dE.p, hdE.size());
    d2h(hinf.data(), infeasible.p, S);
    sync();
    for (int k = 0; k < S; ++k) {
      if (!pending[k]) continue;
      int pick = -1;
      for (int j = 0; j < kTrials; ++j) {
        const double a = std::ldexp(base[k], -j);
        if (a < 1e-12) break;
        if (!((hinf[k] >> j) & 1) && hdE[kTrials * k + j] <= 0.0) {
          pick = j;
          break;
        }
      }
      if (pick >= 0) {
        alpha_h[k] = std::ldexp(base[k], -pick);
        halvings[k] += pick;
        pending[k] = 0;
        --npending;
      } else {
        halvings[k] += kTrials;
        base[k] = std::ldexp(base[k], -kTrials);
        if (base[k] < 1e-12) {
          ls_fail[k] = 1;
          pending[k] = 0;
          --npending;
        }
      }
    }
  }
  h2d(alpha.p, alpha_h.data(), S);
  launch_update(V, dx.p, alpha.p, s);
  for (int k = 0; k < S; ++k)
    if (act_host[k]) prev_alpha[k] = alpha_h[k];
  phase_end(5);
}

// Start of a step for the scenes of mask (all when NULL): targets, prediction, the jump of the
// moving Dirichlet vertices (infeasible_target flags scenes whose jump collides or inverts),
// body penalties reset, start-of-step body residuals, and the bodies already on their target
// snapped (snapped_host).
void Batch::Impl::begin_step(const taccel_targets* tg, const int* mask,
                             std::vector<int>& infeasible_target, std::vector<char>& snapped_host) {
  hipStream_t s = stream();
  View V = view();
  // ---- targets: body y* (host conversion of the public affine maps), moving vertices
  std::vector<double> hstar(12 * (size_t)Nb, 0.0);
  std::vector<double> hmove;
  std::vector<int> hmove_nodes;
  int bglob = 0;
  for (int k = 0; k < S; ++k) {
    const HostScene& H = hs[k];
    if (mask && !mask[k]) {  // scene not stepped this call
      bglob += H.nb;
      continue;
    }
    for (int b = 0; b < H.nb; ++b, ++bglob) {
      const HostBody& hb = H.bodies[b];
      if (!hb.prescribed) continue;
      if (!tg || !tg[k].body_targets)
        throw ApiError(TACCEL_ERR_ARG, "scene " + std::to_string(k) + " has a prescribed body but no body_targets");
      const double* q = tg[k].body_targets + 12 * b;
      const double* A = q + 3;
      double* y = hstar.data() + 12 * (size_t)bglob;
      for (int i = 0; i < 3; ++i) {
        double acc = q[i];
        for (int j = 0; j < 3; ++j) acc += A[3 * i + j] * hb.com0[j];
        y[i] = acc;
      }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) y[3 + 3 * j + i] = A[3 * i + j];
    }
    if (H.n_moving > 0) {
      if (!tg || !tg[k].dirichlet_targets)
        throw ApiError(TACCEL_ERR_ARG, "scene " + std::to_string(k) + " has moving vertices but no dirichlet_targets");
      for (int i = 0; i < 3 * H.n_moving; ++i) hmove.push_back(tg[k].dirichlet_targets[i]);
      for (int v : H.moving) hmove_nodes.push_back(H.node0 + v);
    }
  }
  xn_valid = false;
  h2d(bstar.p, hstar.data(), hstar.size());
  launch_predict(V, s);
  xn_valid = true;
  nfric = 0;
  if (any_fric) build_friction(mask);
  infeasible_target.assign(S, 0);
  if (!hmove_nodes.empty()) {
    mv_nodes.upload(&mem, hmove_nodes);
    mv_tgt.upload(&mem, hmove);
    // The prescribed vertices jump to their targets; the jump must be collision-free and
    // keep every tet positive (INFEASIBLE_TARGET otherwise).  Positions after the jump are
    // staged in r (free at this point).
    HIPCHECK(hipMemcpyAsync(r.p, x.p, sizeof(double) * 3 * (size_t)Nn, hipMemcpyDeviceToDevice, s));
    launch_set_moving(r.p, (int)hmove_nodes.size(), mv_nodes.p, mv_tgt.p, s);
    launch_cpos(V, s);
    launch_cmap(V, r.p, cend.p, s);
    launch_diff3(3 * Ncv, cend.p, cpos.p, cdisp.p, s);
    std::vector<int> all_on(S, 1);
    for (int k = 0; k < S; ++k) all_on[k] = (!mask || mask[k]) && hs[k].n_moving > 0;
    h2d(act.p, all_on.data(), S);
    const int nsw = broad_phase(cpos.p, cend.p, 0, sq, st);
    unsigned long long* amin = u64s.p + S;
    {
      std::vector<unsigned long long> one(S);
      const double d1 = 1.0;
      unsigned long long b1;
      std::memcpy(&b1, &d1, sizeof(double));
      std::fill(one.begin(), one.end(), b1);
      h2d(amin, one.data(), S);
    }
    launch_ccd(V, nsw, sq.p, st.p, amin, s);
    zero(bad.p, sizeof(int) * S);
    launch_tets_positive(V, r.p, bad.p, s);
    std::vector<unsigned long long> ha(S);
    std::vector<int> hb(S);
    d2h(ha.data(), amin, S);
    d2h(hb.data(), bad.p, S);
    sync();
    for (int k = 0; k < S; ++k) {
      double a;
      std::memcpy(&a, &ha[k], sizeof(double));
      infeasible_target[k] = hs[k].n_moving > 0 && (a < 1.0 || hb[k]);
    }
    launch_set_moving(x.p, (int)hmove_nodes.size(), mv_nodes.p, mv_tgt.p, s);
  }
  launch_body_reset(V, 1e6, s);
  cover_valid = false;
  // initial residual of every prescribed body
  unsigned long long* bres = u64s.p + 2 * S;
  zero(bres, sizeof(unsigned long long) * (Nb + 1));
  launch_body_resid(V, bres, s);
  std::vector<unsigned long long> hres(Nb + 1);
  d2h(hres.data(), bres, Nb);
  sync();
  bglob = 0;
  for (auto& H : hs)
    for (auto& hb : H.bodies) {
      double r;
      std::memcpy(&r, &hres[bglob++], sizeof(double));
      hb.r0 = hb.rprev = r;
    }
  // a prescribed body already on its target (zero residual) is snapped before the first Newton
  // iteration: its constraint holds, and the relative snap test could never accept it
  snapped_host.assign(Nb, 0);
  {
    std::vector<int> held(Nb, 0);
    bool any_held = false;
    bglob = 0;
    for (int k = 0; k < S; ++k)
      for (int b = 0; b < hs[k].nb; ++b, ++bglob) {
        const HostBody& hb = hs[k].bodies[b];
        if (hb.prescribed && hb.r0 == 0.0 && (!mask || mask[k])) {
          held[bglob] = 1;
          snapped_host[bglob] = 1;
          any_held = true;
        }
      }
    if (any_held) {
      h2d(action.p, held.data(), Nb);
      launch_al_apply(V, action.p, s);
    }
  }
}

taccel_status Batch::Impl::step(const taccel_targets* tg, taccel_status* per_scene,
                                taccel_step_stats* stats, const int* mask) {
  const auto t_start = std::chrono::steady_clock::now();
  hipStream_t s = stream();
  View V = view();
  std::vector<int> infeasible_target;
  std::vector<char> snapped_host;
  begin_step(tg, mask, infeasible_target, snapped_host);
  unsigned long long* bres = u64s.p + 2 * S;
  std::vector<unsigned long long> hres(Nb + 1);
  int bglob = 0;
  std::fill(prev_alpha.begin(), prev_alpha.end(), 0.0);
  std::fill(gg_prev_h.begin(), gg_prev_h.end(), -1.0);  // every Newton loop starts afresh
  // ---- per-scene state machine
  enum { kNewton = 0, kDone = 1, kFailed = 2 };
  std::vector<int> phase(S, kNewton), status(S, TACCEL_OK), nit(S, 0), tot_nit(S, 0), rounds(S, 1);
  for (int k = 0; k < S; ++k) {
    if (infeasible_target[k]) {
      phase[k] = kFailed;
      status[k] = TACCEL_INFEASIBLE_TARGET;
    }
    if (mask && !mask[k]) phase[k] = kDone;
  }
  std::vector<int> tot_pcg(S, 0), nact_last(S, 0), tot_halv(S, 0);
  std::vector<int> last(S), lsf(S), nanf(S), pcg_it(S), nact(S), halv(S);
  std::vector<int> hact(S);
  int guard = 0;
  for (;;) {
    int nactive = 0;
    for (int k = 0; k < S; ++k) {
      hact[k] = phase[k] == kNewton;
      nactive += hact[k];
    }
    if (nactive == 0) break;
    if (++guard > 1000000) throw ApiError(TACCEL_ERR_HIP, "internal: step state machine did not terminate");
    h2d(act.p, hact.data(), S);
    act_host = hact;
    newton_iteration(last, lsf, nanf, pcg_it, nact, halv);
    std::vector<int> al_scene(S, 0);
    bool any_al = false;
    for (int k = 0; k < S; ++k) {
      if (!hact[k]) continue;
      ++nit[k];
      ++tot_nit[k];
      tot_pcg[k] += pcg_it[k];
      tot_halv[k] += halv[k];
      nact_last[k] = nact[k];
      if (nanf[k]) { phase[k] = kFailed; status[k] = TACCEL_NAN; continue; }
      if (lsf[k]) { phase[k] = kFailed; status[k] = TACCEL_LINESEARCH_FAILED; continue; }
      if (last[k]) {
        al_scene[k] = 1;
        any_al = true;
      } else if (nit[k] >= hs[k].max_newton) {
        phase[k] = kFailed;
        status[k] = TACCEL_NOT_CONVERGED;
      }
    }
    if (!any_al) continue;
    // ---- augmented Lagrangian round for the scenes whose Newton loop converged
    std::vector<int> pending_scene(S, 0);
    std::vector<int> candidates(Nb, 0), actions(Nb, 0);
    bool any_cand = false;
    zero(bres, sizeof(unsigned long long) * (Nb + 1));
    launch_body_resid(V, bres, s);
    d2h(hres.data(), bres, Nb);
    sync();
    bglob = 0;
    for (int k = 0; k < S; ++k)
      for (int b = 0; b < hs[k].nb; ++b, ++bglob) {
        HostBody& hb = hs[k].bodies[b];
        if (!al_scene[k] || !hb.prescribed || snapped_host[bglob]) continue;
        pending_scene[k] = 1;
        double rr;
        std::memcpy(&rr, &hres[bglob], sizeof(double));
        if (rr <= 1e-3 * hb.r0) {
          candidates[bglob] = 1;
          any_cand = true;
        }
        actions[bglob] = rr > 0.5 * hb.rprev ? 3 : 2;
        hb.rprev = rr;
      }
    if (any_cand) {
      // collision-free snap test: move the candidate bodies onto their targets
      std::vector<int> snap_act(S, 0);
      bglob = 0;
      for (int k = 0; k < S; ++k)
        for (int b = 0; b < hs[k].nb; ++b, ++bglob)
          if (candidates[bglob]) snap_act[k] = 1;
      h2d(act.p, snap_act.data(), S);
      h2d(snapcand.p, candidates.data(), Nb);
      launch_cpos(V, s);
      launch_snap_disp(V, snapcand.p, s);
      launch_cend(V, cend.p, s);
      const int nsw = broad_phase(cpos.p, cend.p, 0, sq, st);
      cover_valid = false;
      unsigned long long* amin = u64s.p + S;
      std::vector<unsigned long long> one(S);
      const double d1 = 1.0;
      unsigned long long b1;
      std::memcpy(&b1, &d1, sizeof(double));
      std::fill(one.begin(), one.end(), b1);
      h2d(amin, one.data(), S);
      launch_ccd(V, nsw, sq.p, st.p, amin, s);
      std::vector<unsigned long long> ha(S);
      d2h(ha.data(), amin, S);
      sync();
      bglob = 0;
      for (int k = 0; k < S; ++k) {
        double a;
        std::memcpy(&a, &ha[k], sizeof(double));
        for (int b = 0; b < hs[k].nb; ++b, ++bglob)
          if (candidates[bglob] && a >= 1.0) {
            actions[bglob] = 1;
            snapped_host[bglob] = 1;
          }
      }
    }
    h2d(action.p, actions.data(), Nb);
    launch_al_apply(V, action.p, s);
    for (int k = 0; k < S; ++k) {
      if (!al_scene[k]) continue;
      if (!pending_scene[k]) {
        phase[k] = kDone;
        continue;
      }
      if (rounds[k] >= hs[k].max_al) {
        phase[k] = kFailed;
        status[k] = TACCEL_AL_FAILED;
        continue;
      }
      ++rounds[k];
      nit[k] = 0;
      prev_alpha[k] = 0.0;  // a new Newton loop starts projected
      gg_prev_h[k] = -1.0;  // and with the loosest forcing term
    }
  }
  // ---- finish: velocities for converged scenes, roll back failed ones
  std::vector<int> ok(S), failed(S);
  for (int k = 0; k < S; ++k) {
    const bool stepped = !mask || mask[k];
    ok[k] = stepped && status[k] == TACCEL_OK;
    failed[k] = stepped && status[k] != TACCEL_OK;
  }
  h2d(okflag.p, ok.data(), S);
  h2d(failflag.p, failed.data(), S);
  launch_velocity(V, okflag.p, s);
  launch_rollback(V, failflag.p, s);
  launch_body_clear_lambda(V, failflag.p, s);
  sync();
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  taccel_status first_bad = TACCEL_OK;
  for (int k = 0; k < S; ++k) {
    if (per_scene) per_scene[k] = (taccel_status)status[k];
    if (stats) {
      stats[k].status = status[k];
      stats[k].newton_iters = tot_nit[k];
      stats[k].al_rounds = rounds[k];
      stats[k].pcg_iters = tot_pcg[k];
      stats[k].n_active = nact_last[k];
      stats[k].ls_halvings = tot_halv[k];
      stats[k].step_ms = ms;
    }
    if (status[k] != TACCEL_OK && first_bad == TACCEL_OK) first_bad = (taccel_status)status[k];
    if (!mask || mask[k]) {
      taccel_step_stats& ls = last_stats[k];
      ls.status = status[k];
      ls.newton_iters = tot_nit[k];
      ls.al_rounds = rounds[k];
      ls.pcg_iters = tot_pcg[k];
      ls.n_active = nact_last[k];
      ls.ls_halvings = tot_halv[k];
      ls.step_ms = ms;
    }
  }
  return first_bad;
}

size_t Batch::Impl::device_bytes() const { return mem.held; }

void Batch::Impl::release_all() {
  if (h_pin) (void)hipHostFree(h_pin);
  h_pin = nullptr;
  // DBuf members free themselves through explicit calls below
}

// ------------------------------------------------------------------ Batch API
taccel_status Batch::create(const taccel_scene_desc* d, int n, const taccel_runtime* rt,
                            Batch** out, std::string& err) {
  Batch* b = new Batch();
  b->impl_ = new Impl();
  b->S_ = n;
  if (rt) {
    b->impl_->mem.rt = *rt;
    b->impl_->mem.stream = (hipStream_t)rt->stream;
  }
  try {
    b->impl_->build(d, n);
  } catch (const ApiError& e) {
    err = e.what();
    const taccel_status st = e.st;
    delete b;
    return st;
  }
  *out = b;
  return TACCEL_OK;
}

taccel_status Batch::validate(const taccel_scene_desc* d, int n, std::string& err) {
  Impl I;
  I.validate_only = true;
  try {
    I.build(d, n);
  } catch (const ApiError& e) {
    err = e.what();
    return e.st;
  }
  return TACCEL_OK;
}

Batch::~Batch() {
  if (!impl_) return;
  Impl& I = *impl_;
  if (!I.device_touched) {  // rejected before any device call
    delete impl_;
    return;
  }
  (void)hipStreamSynchronize(I.mem.stream);
  if (I.mem.side) (void)hipStreamSynchronize(I.mem.side);
  if (I.mem.side2) (void)hipStreamSynchronize(I.mem.side2);
  I.release_all();
  for (hipEvent_t e : I.ev_pool) (void)hipEventDestroy(e);
  if (I.ev_fork) (void)hipEventDestroy(I.ev_fork);
  if (I.ev_join) (void)hipEventDestroy(I.ev_join);
  if (I.ev_join2) (void)hipEventDestroy(I.ev_join2);
  if (I.pcg_exec) (void)hipGraphExecDestroy(I.pcg_exec);
  for (hipGraph_t g0 : I.pcg_graphs) (void)hipGraphDestroy(g0);
#define FREE_ALL(...) for (auto* bptr : {__VA_ARGS__}) bptr->free();
  FREE_ALL(&I.x, &I.xn, &I.xhat, &I.v, &I.mass, &I.Dminv, &I.tvol, &I.val, &I.bmass,
           &I.bvol, &I.bstar, &I.blam, &I.bkap, &I.bgrad, &I.bhess, &I.bpinv, &I.cvx, &I.cpos, &I.cdisp,
           &I.cend, &I.elen2, &I.bp_tbox, &I.pmeps, &I.pg, &I.ph, &I.hcoef, &I.gcoef, &I.dval, &I.g, &I.r,
           &I.z, &I.p, &I.p1, &I.q, &I.dx, &I.pinv, &I.P_pq, &I.P_rz0, &I.P_rz1, &I.P_gg, &I.abase,
           &I.alpha, &I.dE, &I.part_nodes, &I.part_tets, &I.e_bodies, &I.e_pairs, &I.part_pairs)
  FREE_ALL(&I.tp_sc, &I.tp_b0, &I.tp_b1, &I.tp_sblk)
  FREE_ALL(&I.fw, &I.fc0, &I.fnrm, &I.fmul, &I.e_fric)
  FREE_ALL(&I.fv, &I.fsoff)
  FREE_ALL(&I.xrest, &I.tac_bary, &I.tac_pos, &I.tac_flow, &I.tac_depth, &I.tac_normal)
  FREE_ALL(&I.tac_nodes, &I.tac_zidx)
  I.tac_zkey.free();
  FREE_ALL(&I.ts_sc, &I.ts_b0, &I.ts_b1, &I.ts_sblk)
  FREE_ALL(&I.cg_blk_agg, &I.cg_agg_b0, &I.cg_agg_b1, &I.cg_sc_a0, &I.cg_sc_m, &I.cg_sc_ts0,
           &I.cg_sc_tsn, &I.cg_sc_tsend, &I.bp_tmp)
  FREE_ALL(&I.cg_d, &I.cg_ainv, &I.cg_rc, &I.P_qc, &I.cg_rca0, &I.cg_rca1, &I.cg_dw, &I.dxc, &I.gres, &I.rpart)
  FREE_ALL(&I.val32, &I.dval32, &I.pinv32, &I.bpinv32, &I.cg_d32, &I.cg_dw32)
  I.fg_prev.free();
  I.cg_sc_off.free();
  FREE_ALL(&I.nfree, &I.nscene, &I.nbody, &I.ntype, &I.tv, &I.tscene, &I.rowptr, &I.col, &I.diag,
           &I.vptr, &I.vlist, &I.bnode, &I.bscene, &I.bpres, &I.bsnap, &I.bcv0, &I.bcv1,
           &I.cvn, &I.cvb, &I.cvfix, &I.cvscene, &I.cvworld, &I.trv, &I.edv, &I.qkind, &I.qidx, &I.qscene,
           &I.act, &I.pdone, &I.exact, &I.indef, &I.tn_sc, &I.tn_b0, &I.tn_b1, &I.tn_sblk, &I.tt_sc, &I.tt_b0, &I.tt_b1,
           &I.tt_sblk, &I.bp_tcell, &I.bp_tncell, &I.bp_toff, &I.bp_bcount, &I.bp_bstart, &I.bp_bfill,
           &I.bp_qcount, &I.bp_qoff, &I.cq, &I.ct, &I.sq, &I.st, &I.cflag, &I.cpos_idx, &I.pkind, &I.pv,
           &I.pscene, &I.hcnt, &I.gcnt, &I.hoff, &I.goff, &I.hidx, &I.gidx, &I.hsrc, &I.gsrc, &I.hidx2,
           &I.gidx2, &I.sflag, &I.segid, &I.segstart, &I.drow, &I.dcol, &I.rowcnt, &I.drowptr, &I.iters,
           &I.bad, &I.infeasible, &I.scnt, &I.cand_off, &I.action, &I.okflag, &I.failflag, &I.snapcand,
           &I.scalars)
  I.hkey.free();
  I.gkey.free();
  I.hkey2.free();
  I.gkey2.free();
  I.u64s.free();
  I.bp_entries.free();
  I.bp_ovf.free();
  I.scratch.free();
  I.mv_nodes.free();
  I.mv_tgt.free();
  I.d_sc.free();
#undef FREE_ALL
  if (I.mem.own_stream) (void)hipStreamDestroy(I.mem.stream);
  if (I.mem.side) (void)hipStreamDestroy(I.mem.side);
  if (I.mem.side2) (void)hipStreamDestroy(I.mem.side2);
  I.mem.side = I.mem.side2 = nullptr;
  delete impl_;
}

taccel_status Batch::step(const taccel_targets* t, taccel_status* per_scene, taccel_step_stats* st,
                          const int* mask) {
  try {
    return impl_->step(t, per_scene, st, mask);
  } catch (const ApiError& e) {
    set_last_error(e.what());
    impl_->discard_pending();
    // roll every scene back to the start of the step (positions saved by the predictor)
    Impl& I = *impl_;
    // (when the error came before the predictor, nothing has been moved yet)
    (void)hipStreamSynchronize(I.mem.stream);
    if (I.mem.side) (void)hipStreamSynchronize(I.mem.side);
    if (I.mem.side2) (void)hipStreamSynchronize(I.mem.side2);
    if (I.xn_valid)
      (void)hipMemcpyAsync(I.x.p, I.xn.p, sizeof(double) * 3 * (size_t)I.Nn, hipMemcpyDeviceToDevice,
                           I.mem.stream);
    (void)hipStreamSynchronize(I.mem.stream);
    if (per_scene)
      for (int k = 0; k < S_; ++k) per_scene[k] = e.st;
    if (st)
      for (int k = 0; k < S_; ++k) {
        std::memset(&st[k], 0, sizeof(st[k]));
        st[k].status = e.st;
      }
    return e.st;
  }
}

static size_t field_count(const Batch::Impl& I, int k, taccel_field f) {
  const HostScene& H = I.hs[k];
  switch (f) {
    case TACCEL_FIELD_X:
    case TACCEL_FIELD_V: return 3 * (size_t)H.nv;
    case TACCEL_FIELD_Q:
    case TACCEL_FIELD_QDOT: return 12 * (size_t)H.nb;
    case TACCEL_FIELD_BODY_X: {
      size_t n = 0;
      for (const auto& b : H.bodies) n += 3 * (size_t)b.nv;
      return n;
    }
    default: break;
  }
  return 0;
}

taccel_status Batch::read(int k, taccel_field f, void* dst, size_t bytes) {
  try {
    Impl& I = *impl_;
    if (k < 0 || k >= S_) throw ApiError(TACCEL_ERR_ARG, "scene index out of range");
    if (f == TACCEL_FIELD_STATS) {
      if (bytes != sizeof(taccel_step_stats) || !dst)
        throw ApiError(TACCEL_ERR_ARG, "state_read: STATS takes one taccel_step_stats");
      std::memcpy(dst, &I.last_stats[k], sizeof(taccel_step_stats));
      return TACCEL_OK;
    }
    if (f == TACCEL_FIELD_CONTACTS) {
      const std::vector<int32_t> c = I.contacts(k);
      if (bytes != c.size() * sizeof(int32_t) || (!c.empty() && !dst))
        throw ApiError(TACCEL_ERR_ARG, "state_read: size mismatch (expected " +
                                           std::to_string(c.size() * sizeof(int32_t)) + " bytes)");
      if (!c.empty()) std::memcpy(dst, c.data(), bytes);
      return TACCEL_OK;
    }
    if (f < TACCEL_FIELD_X || f > TACCEL_FIELD_BODY_X) throw ApiError(TACCEL_ERR_ARG, "unknown field");
    const size_t cnt = field_count(I, k, f);
    if (bytes != cnt * sizeof(double) || (cnt && !dst))
      throw ApiError(TACCEL_ERR_ARG, "state_read: size mismatch (expected " + std::to_string(cnt * 8) + " bytes)");
    const HostScene& H = I.hs[k];
    double* out = static_cast<double*>(dst);
    if (f == TACCEL_FIELD_X || f == TACCEL_FIELD_V) {
      std::vector<double> tmp(cnt);
      I.d2h(tmp.data(), (f == TACCEL_FIELD_X ? I.x.p : I.v.p) + 3 * (size_t)H.node0, cnt);
      I.sync();
      for (int u = 0; u < H.nv; ++u)
        for (int c = 0; c < 3; ++c) out[3 * (size_t)u + c] = tmp[3 * (size_t)H.perm[u] + c];
      return TACCEL_OK;
    }
    const int n_soft_pad = (H.nv + 3) / 4 * 4;
    std::vector<double> y(12 * (size_t)H.nb);
    I.d2h(y.data(), (f == TACCEL_FIELD_QDOT ? I.v.p : I.x.p) + 3 * (size_t)(H.node0 + n_soft_pad), y.size());
    I.sync();
    size_t o = 0;
    for (int b = 0; b < H.nb; ++b) {
      const HostBody& hb = H.bodies[b];
      const double* yb = y.data() + 12 * b;
      double A[9];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[3 * i + j] = yb[3 + 3 * j + i];
      if (f == TACCEL_FIELD_BODY_X) {
        for (int v = 0; v < hb.nv; ++v)
          for (int c = 0; c < 3; ++c) {
            double acc = yb[c];
            for (int j = 0; j < 3; ++j) acc += hb.xbar[3 * v + j] * yb[3 + 3 * j + c];
            out[o++] = acc;
          }
        continue;
      }
      double* qo = out + 12 * b;
      for (int i = 0; i < 3; ++i) {
        double acc = yb[i];
        for (int j = 0; j < 3; ++j) acc -= A[3 * i + j] * hb.com0[j];
        qo[i] = acc;
      }
      for (int m = 0; m < 9; ++m) qo[3 + m] = A[m];
    }
    return TACCEL_OK;
  } catch (const ApiError& e) {
    set_last_error(e.what());
    impl_->discard_pending();
    return e.st;
  }
}

taccel_status Batch::field_bytes(int k, taccel_field f, size_t* bytes) {
  try {
    Impl& I = *impl_;
    if (k < 0 || k >= S_) throw ApiError(TACCEL_ERR_ARG, "scene index out of range");
    if (!bytes) throw ApiError(TACCEL_ERR_ARG, "state_bytes: NULL output");
    if (f == TACCEL_FIELD_STATS) *bytes = sizeof(taccel_step_stats);
    else if (f == TACCEL_FIELD_CONTACTS) *bytes = I.contacts(k).size() * sizeof(int32_t);
    else if (f >= TACCEL_FIELD_X && f <= TACCEL_FIELD_BODY_X) *bytes = field_count(I, k, f) * sizeof(double);
    else throw ApiError(TACCEL_ERR_ARG, "unknown field");
    return TACCEL_OK;
  } catch (const ApiError& e) {
    set_last_error(e.what());
    impl_->discard_pending();
    return e.st;
  }
}

taccel_status Batch::read_device(int k, taccel_field f, void* dst, size_t bytes) {
  try {
    Impl& I = *impl_;
    if (k < 0 || k >= S_) throw ApiError(TACCEL_ERR_ARG, "scene index out of range");
    if (f < TACCEL_FIELD_X || f > TACCEL_FIELD_BODY_X)
      throw ApiError(TACCEL_ERR_ARG, "read_device: fields X, V, Q, QDOT and BODY_X only");
    const size_t cnt = field_count(I, k, f);
    if (bytes != cnt * sizeof(double) || (cnt && !dst))
      throw ApiError(TACCEL_ERR_ARG, "read_device: size mismatch (expected " + std::to_string(cnt * 8) + " bytes)");
    if (cnt == 0) return TACCEL_OK;
    const HostScene& H = I.hs[k];
    hipStream_t s = I.stream();
    double* out = static_cast<double*>(dst);
    DBuf<int> idx;
    DBuf<double> com;
    if (f == TACCEL_FIELD_X || f == TACCEL_FIELD_V || f == TACCEL_FIELD_BODY_X) {
      std::vector<int> h;
      if (f == TACCEL_FIELD_BODY_X) {
        // body vertices in world order -> their contact vertices
        std::vector<int> cv_of(H.cv_world.size() + (size_t)H.nv, -1);
        for (size_t li = 0; li < H.cv_world.size(); ++li) {
          const int w = H.cv_world[li];
          if (w >= H.nv) cv_of[w - H.nv] = H.cv0 + (int)li;
        }
        for (size_t i = 0; i < cnt / 3; ++i) {
          if (cv_of[i] < 0) throw ApiError(TACCEL_ERR_ARG, "read_device: body vertex without contact vertex");
          h.push_back(cv_of[i]);
        }
        launch_cpos(I.view(), s);
      } else {
        for (int u = 0; u < H.nv; ++u) h.push_back(H.node0 + H.perm[u]);
      }
      idx.upload(&I.mem, h);
      const double* src = f == TACCEL_FIELD_X ? I.x.p : f == TACCEL_FIELD_V ? I.v.p : I.cpos.p;
      launch_gather3((int)h.size(), idx.p, src, out, s);
    } else {
      std::vector<double> c0(3 * (size_t)H.nb);
      for (int b = 0; b < H.nb; ++b)
        for (int j = 0; j < 3; ++j) c0[3 * b + j] = H.bodies[b].com0[j];
      com.upload(&I.mem, c0);
      const int n_soft_pad = (H.nv + 3) / 4 * 4;
      const double* y = (f == TACCEL_FIELD_QDOT ? I.v.p : I.x.p) + 3 * (size_t)(H.node0 + n_soft_pad);
      launch_body_public(H.nb, y, com.p, out, s);
    }
    I.sync();
    idx.free();
    com.free();
    return TACCEL_OK;
  } catch (const ApiError& e) {
    set_last_error(e.what());
    impl_->discard_pending();
    return e.st;
  }
}

taccel_status Batch::debug_system(const taccel_targets* tg, double* grad, int32_t* brow_out,
                                  int32_t* bcol_out, double* bval_out, int32_t cap,
                                  int32_t* n_blocks) {
  Impl& I = *impl_;
  bool begun = false;
  // the scene goes back to the start of the step whatever happens after begin_step
  auto restore = [&]() {
    if (!begun) return;
    begun = false;
    View V = I.view();
    const int one = 1;
    I.h2d(I.failflag.p, &one, 1);
    launch_rollback(V, I.failflag.p, I.stream());
    launch_body_clear_lambda(V, I.failflag.p, I.stream());
    I.cover_valid = false;
    I.sync();
  };
  try {
    if (I.S != 1) throw ApiError(TACCEL_ERR_ARG, "debug_system works on a single scene");
    if (!n_blocks || (cap > 0 && (!brow_out || !bcol_out || !bval_out)))
      throw ApiError(TACCEL_ERR_ARG, "debug_system: NULL output");
    const HostScene& H = I.hs[0];
    std::vector<int> infeasible;
    std::vector<char> snapped;
    begun = true;
    I.begin_step(tg, nullptr, infeasible, snapped);
    if (infeasible[0]) throw ApiError(TACCEL_INFEASIBLE_TARGET, "debug_system: infeasible targets");
    // the first Newton iteration of the step: projected Hessians, a fresh broad phase
    I.act_host.assign(1, 1);
    I.h2d(I.act.p, I.act_host.data(), 1);
    I.exact_h.assign(1, 0);
    I.h2d(I.exact.p, I.exact_h.data(), 1);
    I.cover_valid = false;
    std::vector<int> bp_bad(1, 0);
    const int np = I.prepare_pairs(bp_bad);
    I.derivatives(np, np + I.nfric);
    const int Nn = I.Nn;
    std::vector<double> g(3 * (size_t)Nn);
    std::vector<int> rp(Nn + 1), drp(Nn + 1), cl(I.nnz), nf(Nn);
    I.d2h(g.data(), I.g.p, g.size());
    I.d2h(rp.data(), I.rowptr.p, rp.size());
    I.d2h(drp.data(), I.drowptr.p, drp.size());
    I.d2h(cl.data(), I.col.p, cl.size());
    I.d2h(nf.data(), I.nfree.p, nf.size());
    I.sync();
    const int ndyn = drp[Nn];
    std::vector<int> dcl(std::max(ndyn, 1));
    std::vector<double> sv(9 * (size_t)I.nnz), dv(9 * (size_t)std::max(ndyn, 1));
    I.d2h(dcl.data(), I.dcol.p, ndyn);
    if (I.mixed) {
      std::vector<float> a(sv.size()), b(dv.size());
      I.d2h(a.data(), reinterpret_cast<const float*>(I.val.p), a.size());
      I.d2h(b.data(), reinterpret_cast<const float*>(I.dval.p), 9 * (size_t)ndyn);
      I.sync();
      for (size_t k = 0; k < a.size(); ++k) sv[k] = a[k];
      for (size_t k = 0; k < 9 * (size_t)ndyn; ++k) dv[k] = b[k];
    } else {
      I.d2h(sv.data(), I.val.p, sv.size());
      I.d2h(dv.data(), I.dval.p, 9 * (size_t)ndyn);
      I.sync();
    }
    restore();
    // internal node -> caller's node (soft vertices in the caller's order, then 4 per body)
    std::vector<int> ext(Nn, -1);
    for (int u = 0; u < H.nv; ++u) ext[H.node0 + H.perm[u]] = u;
    const int npad = (H.nv + 3) / 4 * 4;
    for (int b = 0; b < H.nb; ++b)
      for (int j = 0; j < 4; ++j) ext[H.node0 + npad + 4 * b + j] = H.nv + 4 * b + j;
    const int next = H.nv + 4 * H.nb;
    if (grad) {
      std::fill(grad, grad + 3 * (size_t)next, 0.0);
      for (int n = 0; n < Nn; ++n)
        if (ext[n] >= 0 && nf[n])
          for (int c = 0; c < 3; ++c) grad[3 * (size_t)ext[n] + c] = g[3 * (size_t)n + c];
    }
    std::vector<std::pair<std::pair<int, int>, std::array<double, 9>>> blocks;
    auto add = [&](int r, int c, const double* v) {
      if (ext[r] < 0 || ext[c] < 0 || !nf[r] || !nf[c]) return;
      std::array<double, 9> a;
      for (int k = 0; k < 9; ++k) a[k] = v[k];
      blocks.push_back({{ext[r], ext[c]}, a});
    };
    for (int r = 0; r < Nn; ++r) {
      for (int k = rp[r]; k < rp[r + 1]; ++k) add(r, cl[k], sv.data() + 9 * (size_t)k);
      for (int k = drp[r]; k < drp[r + 1]; ++k) add(r, dcl[k], dv.data() + 9 * (size_t)k);
    }
    std::sort(blocks.begin(), blocks.end(),
              [](const auto& a, const auto& b) { return a.first < b.first; });
    int nb = 0;
    for (size_t k = 0; k < blocks.size(); ++k) {
      if (nb > 0 && blocks[k].first == blocks[k - 1].first) {
        if (nb <= cap)
          for (int e = 0; e < 9; ++e) bval_out[9 * (size_t)(nb - 1) + e] += blocks[k].second[e];
        continue;
      }
      if (nb < cap) {
        brow_out[nb] = blocks[k].first.first;
        bcol_out[nb] = blocks[k].first.second;
        for (int e = 0; e < 9; ++e) bval_out[9 * (size_t)nb + e] = blocks[k].second[e];
      }
      ++nb;
    }
    *n_blocks = nb;
    return TACCEL_OK;
  } catch (const ApiError& e) {
    set_last_error(e.what());
    impl_->discard_pending();
    try {
      restore();
    } catch (const ApiError&) {
    }
    return e.st;
  }
}

taccel_status Batch::export_state(int k, SceneState& out) {
  try {
    Impl& I = *impl_;
    if (k < 0 || k >= S_) throw ApiError(TACCEL_ERR_ARG, "scene index out of range");
    const size_t n0 = I.hs[k].node0, n1 = I.hs[k].node1;
    const size_t b0 = I.hsc[k].body0, b1 = I.hsc[k].body1;
    out.x.resize(3 * (n1 - n0));
    out.v.resize(3 * (n1 - n0));
    out.lam.resize(12 * (b1 - b0));
    I.d2h(out.x.data(), I.x.p + 3 * n0, out.x.size());
    I.d2h(out.v.data(), I.v.p + 3 * n0, out.v.size());
    I.d2h(out.lam.data(), I.blam.p + 12 * b0, out.lam.size());
    I.sync();
    return TACCEL_OK;
  } catch (const ApiError& e) {
    set_last_error(e.what());
    impl_->discard_pending();
    return e.st;
  }
}

taccel_status Batch::import_state(int k, const SceneState& in) {
  try {
    Impl& I = *impl_;
    if (k < 0 || k >= S_) throw ApiError(TACCEL_ERR_ARG, "scene index out of range");
    const size_t n0 = I.hs[k].node0, n1 = I.hs[k].node1;
    const size_t b0 = I.hsc[k].body0, b1 = I.hsc[k].body1;
    if (in.x.size() != 3 * (n1 - n0) || in.v.size() != 3 * (n1 - n0) || in.lam.size() != 12 * (b1 - b0))
      throw ApiError(TACCEL_ERR_ARG, "import_state: the state is of another scene");
    I.h2d(I.x.p + 3 * n0, in.x.data(), in.x.size());
    I.h2d(I.v.p + 3 * n0, in.v.data(), in.v.size());
    I.h2d(I.blam.p + 12 * b0, in.lam.data(), in.lam.size());
    I.cover_valid = false;
    I.sync();
    return TACCEL_OK;
  } catch (const ApiError& e) {
    set_last_error(e.what());
    impl_->discard_pending();
    return e.st;
  }
}

taccel_status Batch::reset(const uint8_t* mask) {
  try {
    Impl& I = *impl_;
    hipStream_t s = I.stream();
    // runs of consecutive selected scenes are contiguous in the node and body arrays
    for (int k = 0; k < S_;) {
      if (mask && !mask[k]) {
        ++k;
        continue;
      }
      int e = k;
      while (e + 1 < S_ && (!mask || mask[e + 1])) ++e;
      const size_t n0 = I.hs[k].node0, n1 = I.hs[e].node1;
      HIPCHECK(hipMemcpyAsync(I.x.p + 3 * n0, I.xrest.p + 3 * n0, sizeof(double) * 3 * (n1 - n0),
                              hipMemcpyDeviceToDevice, s));
      I.zero(I.v.p + 3 * n0, sizeof(double) * 3 * (n1 - n0));
      const size_t b0 = I.hsc[k].body0, b1 = I.hsc[e].body1;
      if (b1 > b0) I.zero(I.blam.p + 12 * b0, sizeof(double) * 12 * (b1 - b0));
      for (int j = k; j <= e; ++j) I.last_stats[j] = taccel_step_stats{};
      k = e + 1;
    }
    I.cover_valid = false;
    I.sync();
    return TACCEL_OK;
  } catch (const ApiError& e) {
    set_last_error(e.what());
    impl_->discard_pending();
    return e.st;
  }
}

taccel_status Batch::write(int k, taccel_field f, const void* src, size_t bytes) {
  try {
    Impl& I = *impl_;
    if (k < 0 || k >= S_) throw ApiError(TACCEL_ERR_ARG, "scene index out of range");
    if (f == TACCEL_FIELD_BODY_X || f == TACCEL_FIELD_CONTACTS || f == TACCEL_FIELD_STATS)
      throw ApiError(TACCEL_ERR_ARG, "field is read-only");
    if (f < TACCEL_FIELD_X || f > TACCEL_FIELD_BODY_X) throw ApiError(TACCEL_ERR_ARG, "unknown field");
    const size_t cnt = field_count(I, k, f);
    if (bytes != cnt * sizeof(double) || (cnt && !src)) throw ApiError(TACCEL_ERR_ARG, "state_write: size mismatch");
    const HostScene& H = I.hs[k];
    const double* in = static_cast<const double*>(src);
    if (f == TACCEL_FIELD_X || f == TACCEL_FIELD_V) {
      std::vector<double> tmp(cnt);
      for (int u = 0; u < H.nv; ++u)
        for (int c = 0; c < 3; ++c) tmp[3 * (size_t)H.perm[u] + c] = in[3 * (size_t)u + c];
      I.h2d((f == TACCEL_FIELD_X ? I.x.p : I.v.p) + 3 * (size_t)H.node0, tmp.data(), cnt);
      I.sync();
      return TACCEL_OK;
    }
    const int n_soft_pad = (H.nv + 3) / 4 * 4;
    std::vector<double> y(12 * (size_t)H.nb);
    for (int b = 0; b < H.nb; ++b) {
      const HostBody& hb = H.bodies[b];
      const double* q = in + 12 * b;
      const double* A = q + 3;
      double* yb = y.data() + 12 * b;
      for (int i = 0; i < 3; ++i) {
        double acc = q[i];
        for (int j = 0; j < 3; ++j) acc += A[3 * i + j] * hb.com0[j];
        yb[i] = acc;
      }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) yb[3 + 3 * j + i] = A[3 * i + j];
    }
    I.h2d((f == TACCEL_FIELD_QDOT ? I.v.p : I.x.p) + 3 * (size_t)(H.node0 + n_soft_pad), y.data(), y.size());
    if (f == TACCEL_FIELD_Q && H.nb > 0) {
      // a new body state: the multipliers carried over from the last step no longer apply
      const std::vector<double> zeros(12 * (size_t)H.nb, 0.0);
      I.h2d(I.blam.p + 12 * (size_t)I.hsc[k].body0, zeros.data(), zeros.size());
    }
    I.sync();
    return TACCEL_OK;
  } catch (const ApiError& e) {
    set_last_error(e.what());
    impl_->discard_pending();
    return e.st;
  }
}

size_t Batch::device_bytes() const { return impl_->device_bytes(); }
void Batch::set_byte_limit(size_t bytes) { impl_->mem.limit = bytes; }

taccel_status Batch::markers(int k, int m, const int32_t* tris, const double* bary, double* pos,
                             double* flow) {
  try {
    Impl& I = *impl_;
    if (k < 0 || k >= S_) throw ApiError(TACCEL_ERR_ARG, "scene index out of range");
    if (m < 0 || (m > 0 && (!tris || !bary || !pos || !flow)))
      throw ApiError(TACCEL_ERR_ARG, "markers: bad arguments");
    if (m == 0) return TACCEL_OK;
    for (int i = 0; i < 3 * m; ++i)
      if (!(bary[i] >= 0.0 && bary[i] <= 1.0)) throw ApiError(TACCEL_ERR_ARG, "markers: barycentric coordinate outside [0, 1]");
    const std::vector<int> nodes = I.soft_nodes(k, 3 * m, tris);
    I.tac_nodes.upload(&I.mem, nodes);
    I.tac_bary.upload(&I.mem, std::vector<double>(bary, bary + 3 * (size_t)m));
    I.tac_pos.ensure(&I.mem, 3 * (size_t)m);
    I.tac_flow.ensure(&I.mem, 3 * (size_t)m);
    launch_markers(m, I.tac_nodes.p, I.tac_bary.p, I.x.p, I.xrest.p, I.tac_pos.p, I.tac_flow.p, I.stream());
    I.d2h(pos, I.tac_pos.p, 3 * (size_t)m);
    I.d2h(flow, I.tac_flow.p, 3 * (size_t)m);
    I.sync();
    return TACCEL_OK;
  } catch (const ApiError& e) {
    set_last_error(e.what());
    impl_->discard_pending();
    return e.st;
  }
}

taccel_status Batch::depth_map(int k, const taccel_camera* cam, int ntri, const int32_t* tris,
                               double* depth, double* normal) {
  try {
    Impl& I = *impl_;
    if (k < 0 || k >= S_) throw ApiError(TACCEL_ERR_ARG, "scene index out of range");
    if (!cam || ntri < 0 || (ntri > 0 && !tris) || !depth || !normal)
      throw ApiError(TACCEL_ERR_ARG, "depth_map: bad arguments");
    if (cam->width <= 0 || cam->height <= 0 || (long long)cam->width * cam->height > (1ll << 26))
      throw ApiError(TACCEL_ERR_ARG, "depth_map: image must have 1 to 2^26 pixels");
    if (!(cam->pixel > 0.0) || !std::isfinite(cam->pixel)) throw ApiError(TACCEL_ERR_ARG, "depth_map: pixel pitch must be > 0");
    Camera c;
    double uu = 0, vv = 0, uv = 0;
    for (int i = 0; i < 3; ++i) {
      c.o[i] = cam->origin[i];
      c.eu[i] = cam->axis_u[i];
      c.ev[i] = cam->axis_v[i];
      uu += c.eu[i] * c.eu[i];
      vv += c.ev[i] * c.ev[i];
      uv += c.eu[i] * c.ev[i];
      if (!std::isfinite(c.o[i])) throw ApiError(TACCEL_ERR_ARG, "depth_map: origin must be finite");
    }
    if (!(std::fabs(uu - 1.0) <= 1e-9 && std::fabs(vv - 1.0) <= 1e-9 && std::fabs(uv) <= 1e-9))
      throw ApiError(TACCEL_ERR_ARG, "depth_map: axis_u and axis_v must be orthonormal");
    // en = eu x ev, one product per statement (no fused multiply-add)
    for (int i = 0; i < 3; ++i) {
      const int a = (i + 1) % 3, b = (i + 2) % 3;
      const double p = c.eu[a] * c.ev[b];
      const double q = c.eu[b] * c.ev[a];
      c.en[i] = p - q;
    }
    c.pix = cam->pixel;
    c.W = cam->width;
    c.H = cam->height;
    const int npix = c.W * c.H;
    const std::vector<int> nodes = I.soft_nodes(k, 3 * ntri, tris);
    hipStream_t s = I.stream();
    I.tac_nodes.upload(&I.mem, nodes.empty() ? std::vector<int>(3, 0) : nodes);
    I.tac_zkey.ensure(&I.mem, npix);
    I.tac_zidx.ensure(&I.mem, npix);
    I.tac_depth.ensure(&I.mem, npix);
    I.tac_normal.ensure(&I.mem, 3 * (size_t)npix);
    launch_depth_clear(npix, I.tac_zkey.p, I.tac_zidx.p, s);
    launch_depth_raster(c, ntri, I.tac_nodes.p, I.x.p, I.tac_zkey.p, I.tac_zidx.p, 0, s);
    launch_depth_raster(c, ntri, I.tac_nodes.p, I.x.p, I.tac_zkey.p, I.tac_zidx.p, 1, s);
    launch_depth_finish(c, I.tac_nodes.p, I.x.p, I.tac_zkey.p, I.tac_zidx.p, I.tac_depth.p, I.tac_normal.p, s);
    I.d2h(depth, I.tac_depth.p, npix);
    I.d2h(normal, I.tac_normal.p, 3 * (size_t)npix);
    I.sync();
    return TACCEL_OK;
  } catch (const ApiError& e) {
    set_last_error(e.what());
    impl_->discard_pending();
    return e.st;
  }
}

taccel_status Batch::debug_candidates(const double* P0, const double* P1, int32_t* out, int32_t cap,
                                      int32_t* n) {
  try {
    Impl& I = *impl_;
    if (I.S != 1) throw ApiError(TACCEL_ERR_ARG, "debug_candidates works on a single scene");
    const HostScene& H = I.hs[0];
    std::vector<double> a(3 * (size_t)I.Ncv), b(3 * (size_t)I.Ncv);
    for (int cv = 0; cv < I.Ncv; ++cv)
      for (int c = 0; c < 3; ++c) {
        a[3 * cv + c] = P0[3 * (size_t)H.cv_world[cv] + c];
        if (P1) b[3 * cv + c] = P1[3 * (size_t)H.cv_world[cv] + c];
      }
    DBuf<double> d0, d1;
    d0.upload(&I.mem, a);
    if (P1) d1.upload(&I.mem, b);
    const int nc = I.broad_phase(d0.p, P1 ? d1.p : nullptr, 1, I.cq, I.ct);
    std::vector<int> hq(std::max(nc, 1)), ht(std::max(nc, 1)), qk(I.Nq), qi(I.Nq), tr(3 * (size_t)I.Ntr),
        ed(2 * (size_t)I.Ned);
    I.d2h(hq.data(), I.cq.p, nc);
    I.d2h(ht.data(), I.ct.p, nc);
    I.d2h(qk.data(), I.qkind.p, I.Nq);
    I.d2h(qi.data(), I.qidx.p, I.Nq);
    I.d2h(tr.data(), I.trv.p, tr.size());
    I.d2h(ed.data(), I.edv.p, ed.size());
    I.sync();
    d0.free();
    d1.free();
    *n = nc;
    for (int k = 0; k < nc && k < cap; ++k) {
      int rec[5];
      const int qq = hq[k], t = ht[k];
      rec[0] = qk[qq];
      if (qk[qq] == 0) {
        rec[1] = H.cv_world[qi[qq]];
        int w[3] = {H.cv_world[tr[3 * t]], H.cv_world[tr[3 * t + 1]], H.cv_world[tr[3 * t + 2]]};
        std::sort(w, w + 3);
        rec[2] = w[0]; rec[3] = w[1]; rec[4] = w[2];
      } else {
        const int e1 = qi[qq];
        int a0 = H.cv_world[ed[2 * e1]], a1 = H.cv_world[ed[2 * e1 + 1]];
        int b0 = H.cv_world[ed[2 * t]], b1 = H.cv_world[ed[2 * t + 1]];
        if (a0 > a1) std::swap(a0, a1);
        if (b0 > b1) std::swap(b0, b1);
        if (std::make_pair(b0, b1) < std::make_pair(a0, a1)) { std::swap(a0, b0); std::swap(a1, b1); }
        rec[1] = a0; rec[2] = a1; rec[3] = b0; rec[4] = b1;
      }
      for (int j = 0; j < 5; ++j) out[5 * k + j] = rec[j];
    }
    return TACCEL_OK;
  } catch (const ApiError& e) {
    set_last_error(e.what());
    impl_->discard_pending();
    return e.st;
  }
}

}  // namespace tc
