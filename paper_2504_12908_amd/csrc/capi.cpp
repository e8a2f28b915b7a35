// C-ABI of the taccel library (declarations and contracts in include/taccel.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dmath.h"
#include "kernels.h"

namespace tc {
const char* last_error_cstr();
}

struct taccel_scene {
  tc::Batch* b;
};
struct taccel_batch {
  tc::Batch* b;
};

namespace {

taccel_status fail(taccel_status s, const std::string& msg) {
  tc::set_last_error(msg);
  return s;
}

// Small RAII device buffer for the evaluators.
struct Dev {
  void* p = nullptr;
  explicit Dev(size_t bytes) {
    if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess) p = nullptr;
  }
  ~Dev() {
    if (p) (void)hipFree(p);
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

taccel_status hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return TACCEL_OK;
  return fail(e == hipErrorOutOfMemory ? TACCEL_ERR_OOM : TACCEL_ERR_HIP,
              std::string(what) + ": " + hipGetErrorString(e));
}

template <class T>
taccel_status fetch(T* host, const Dev& d, size_t n) {
  if (!host) return TACCEL_OK;
  return hip_status(hipMemcpy(host, d.p, sizeof(T) * n, hipMemcpyDeviceToHost), "hipMemcpy D2H");
}

}  // namespace

extern "C" {

const char* taccel_last_error(void) { return tc::last_error_cstr(); }

const char* taccel_status_str(taccel_status s) {
  switch (s) {
    case TACCEL_OK: return "OK";
    case TACCEL_ERR_ARG: return "ERR_ARG";
    case TACCEL_ERR_HIP: return "ERR_HIP";
    case TACCEL_NOT_CONVERGED: return "NOT_CONVERGED";
    case TACCEL_LINESEARCH_FAILED: return "LINESEARCH_FAILED";
    case TACCEL_AL_FAILED: return "AL_FAILED";
    case TACCEL_NAN: return "NAN";
    case TACCEL_INFEASIBLE_TARGET: return "INFEASIBLE_TARGET";
    case TACCEL_ERR_OOM: return "ERR_OOM";
    case TACCEL_INFEASIBLE: return "INFEASIBLE";
    case TACCEL_CANCELLED: return "CANCELLED";
  }
  return "UNKNOWN";
}

taccel_status taccel_batch_create(const taccel_scene_desc* descs, int32_t n, const taccel_runtime* rt,
                                  taccel_batch** out) {
  if (!descs || n <= 0 || !out) return fail(TACCEL_ERR_ARG, "batch_create: descs, n > 0 and out required");
  *out = nullptr;
  tc::Batch* b = nullptr;
  std::string err;
  const taccel_status st = tc::Batch::create(descs, n, rt, &b, err);
  if (st != TACCEL_OK) return fail(st, err);
  *out = new (std::nothrow) taccel_batch{b};
  if (!*out) {
    delete b;
    return fail(TACCEL_ERR_OOM, "host allocation failed");
  }
  return TACCEL_OK;
}

taccel_status taccel_batch_step(taccel_batch* b, const taccel_targets* targets, taccel_status* per_scene,
                                taccel_step_stats* stats) {
  if (!b) return fail(TACCEL_ERR_ARG, "batch_step: NULL batch");
  return b->b->step(targets, per_scene, stats);
}

taccel_status taccel_batch_read(const taccel_batch* b, int32_t scene, taccel_field f, void* dst, size_t bytes) {
  if (!b) return fail(TACCEL_ERR_ARG, "batch_read: NULL batch");
  return b->b->read(scene, f, dst, bytes);
}

taccel_status taccel_batch_write(taccel_batch* b, int32_t scene, taccel_field f, const void* src, size_t bytes) {
  if (!b) return fail(TACCEL_ERR_ARG, "batch_write: NULL batch");
  return b->b->write(scene, f, src, bytes);
}

taccel_status taccel_batch_state_bytes(const taccel_batch* b, int32_t scene, taccel_field f, size_t* bytes) {
  if (!b) return fail(TACCEL_ERR_ARG, "batch_state_bytes: NULL batch");
  return b->b->field_bytes(scene, f, bytes);
}

taccel_status taccel_batch_read_device(const taccel_batch* b, int32_t scene, taccel_field f, void* dst,
                                       size_t bytes) {
  if (!b) return fail(TACCEL_ERR_ARG, "batch_read_device: NULL batch");
  return b->b->read_device(scene, f, dst, bytes);
}

taccel_status taccel_batch_reset(taccel_batch* b, const uint8_t* mask) {
  if (!b) return fail(TACCEL_ERR_ARG, "batch_reset: NULL batch");
  return b->b->reset(mask);
}

void taccel_batch_destroy(taccel_batch* b) {
  if (!b) return;
  delete b->b;
  delete b;
}

taccel_status taccel_batch_markers(const taccel_batch* b, int32_t scene, int32_t m, const int32_t* tris,
                                   const double* bary, double* pos, double* flow) {
  if (!b) return fail(TACCEL_ERR_ARG, "batch_markers: NULL batch");
  return b->b->markers(scene, m, tris, bary, pos, flow);
}

taccel_status taccel_batch_depth_map(const taccel_batch* b, int32_t scene, const taccel_camera* cam,
                                     int32_t ntri, const int32_t* tris, double* depth, double* normal) {
  if (!b) return fail(TACCEL_ERR_ARG, "batch_depth_map: NULL batch");
  return b->b->depth_map(scene, cam, ntri, tris, depth, normal);
}

taccel_status taccel_markers(const taccel_scene* s, int32_t m, const int32_t* tris, const double* bary,
                             double* pos, double* flow) {
  if (!s) return fail(TACCEL_ERR_ARG, "markers: NULL scene");
  return s->b->markers(0, m, tris, bary, pos, flow);
}

taccel_status taccel_depth_map(const taccel_scene* s, const taccel_camera* cam, int32_t ntri,
                               const int32_t* tris, double* depth, double* normal) {
  if (!s) return fail(TACCEL_ERR_ARG, "depth_map: NULL scene");
  return s->b->depth_map(0, cam, ntri, tris, depth, normal);
}

taccel_status taccel_scene_create(const taccel_scene_desc* d, const taccel_runtime* rt, taccel_scene** out) {
  if (!d || !out) return fail(TACCEL_ERR_ARG, "scene_create: desc and out required");
  *out = nullptr;
  tc::Batch* b = nullptr;
  std::string err;
  const taccel_status st = tc::Batch::create(d, 1, rt, &b, err);
  if (st != TACCEL_OK) return fail(st, err);
  *out = new (std::nothrow) taccel_scene{b};
  if (!*out) {
    delete b;
    return fail(TACCEL_ERR_OOM, "host allocation failed");
  }
  return TACCEL_OK;
}

taccel_status taccel_step(taccel_scene* s, const taccel_targets* targets, taccel_step_stats* stats) {
  if (!s) return fail(TACCEL_ERR_ARG, "step: NULL scene");
  taccel_status per;
  return s->b->step(targets, &per, stats);
}

taccel_status taccel_state_read(const taccel_scene* s, taccel_field f, void* dst, size_t bytes) {
  if (!s) return fail(TACCEL_ERR_ARG, "state_read: NULL scene");
  return s->b->read(0, f, dst, bytes);
}

taccel_status taccel_state_write(taccel_scene* s, taccel_field f, const void* src, size_t bytes) {
  if (!s) return fail(TACCEL_ERR_ARG, "state_write: NULL scene");
  return s->b->write(0, f, src, bytes);
}

taccel_status taccel_state_bytes(const taccel_scene* s, taccel_field f, size_t* bytes) {
  if (!s) return fail(TACCEL_ERR_ARG, "state_bytes: NULL scene");
  return s->b->field_bytes(0, f, bytes);
}

taccel_status taccel_state_read_device(const taccel_scene* s, taccel_field f, void* dst, size_t bytes) {
  if (!s) return fail(TACCEL_ERR_ARG, "state_read_device: NULL scene");
  return s->b->read_device(0, f, dst, bytes);
}

taccel_status taccel_scene_reset(taccel_scene* s) {
  if (!s) return fail(TACCEL_ERR_ARG, "scene_reset: NULL scene");
  return s->b->reset(nullptr);
}

void taccel_scene_destroy(taccel_scene* s) {
  if (!s) return;
  delete s->b;
  delete s;
}

taccel_status taccel_debug_system(taccel_scene* s, const taccel_targets* t, double* grad,
                                  int32_t* brow, int32_t* bcol, double* bval, int32_t cap,
                                  int32_t* n_blocks) {
  if (!s) return fail(TACCEL_ERR_ARG, "debug_system: NULL scene");
  return s->b->debug_system(t, grad, brow, bcol, bval, cap, n_blocks);
}

taccel_status taccel_debug_candidates(taccel_scene* s, const double* P0, const double* P1, int32_t* out,
                                      int32_t cap, int32_t* n) {
  if (!s || !P0 || !n || (cap > 0 && !out)) return fail(TACCEL_ERR_ARG, "debug_candidates: bad arguments");
  return s->b->debug_candidates(P0, P1, out, cap, n);
}

taccel_status taccel_debug_fem(int32_t n, const double* rest, const double* x, double youngs, double poisson,
                               double* e, double* g, double* H, double* Hp) {
  if (n < 0 || (n > 0 && (!rest || !x))) return fail(TACCEL_ERR_ARG, "debug_fem: bad arguments");
  if (n == 0) return TACCEL_OK;
  std::vector<double> Dminv(9 * (size_t)n), vol(n);
  for (int t = 0; t < n; ++t) {
    const double* r = rest + 12 * (size_t)t;
    double Dm[9];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) Dm[3 * i + k] = r[3 * (k + 1) + i] - r[i];
    const double det = tc::det3(Dm);
    if (!(det > 0.0)) return fail(TACCEL_ERR_ARG, "debug_fem: inverted rest tet");
    double C[9];
    tc::cofactor3(Dm, C);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Dminv[9 * (size_t)t + 3 * i + j] = C[3 * j + i] / det;
    vol[t] = det / 6.0;
  }
  const double mu = youngs / (2.0 * (1.0 + poisson));
  const double lam = youngs * poisson / ((1.0 + poisson) * (1.0 - 2.0 * poisson));
  Dev dx(sizeof(double) * 12 * n), dD(sizeof(double) * 9 * n), dv(sizeof(double) * n);
  Dev de(sizeof(double) * n), dg(sizeof(double) * 12 * n), dH(sizeof(double) * 144 * n),
      dHp(sizeof(double) * 144 * n);
  if (!dx.p || !dD.p || !dv.p || !de.p || !dg.p || !dH.p || !dHp.p) return fail(TACCEL_ERR_OOM, "debug_fem: hipMalloc");
  taccel_status st;
  if ((st = hip_status(hipMemcpy(dx.p, x, sizeof(double) * 12 * n, hipMemcpyHostToDevice), "H2D")) != TACCEL_OK) return st;
  if ((st = hip_status(hipMemcpy(dD.p, Dminv.data(), sizeof(double) * 9 * n, hipMemcpyHostToDevice), "H2D")) != TACCEL_OK) return st;
  if ((st = hip_status(hipMemcpy(dv.p, vol.data(), sizeof(double) * n, hipMemcpyHostToDevice), "H2D")) != TACCEL_OK) return st;
  tc::launch_debug_fem(n, dx.as<double>(), dD.as<double>(), dv.as<double>(), mu, lam, de.as<double>(),
                       dg.as<double>(), dH.as<double>(), dHp.as<double>(), nullptr);
  if ((st = hip_status(hipDeviceSynchronize(), "debug_fem kernel")) != TACCEL_OK) return st;
  if ((st = fetch(e, de, n)) != TACCEL_OK) return st;
  if ((st = fetch(g, dg, 12 * (size_t)n)) != TACCEL_OK) return st;
  if ((st = fetch(H, dH, 144 * (size_t)n)) != TACCEL_OK) return st;
  return fetch(Hp, dHp, 144 * (size_t)n);
}

taccel_status taccel_debug_barrier(int32_t n, const int32_t* kinds, const double* x, const double* meps,
                                   double dhat, double kappa, double* e, double* g, double* H, double* Hp,
                                   int32_t* types) {
  if (n < 0 || (n > 0 && (!kinds || !x || !meps))) return fail(TACCEL_ERR_ARG, "debug_barrier: bad arguments");
  if (n == 0) return TACCEL_OK;
  for (int k = 0; k < n; ++k)
    if (kinds[k] != 0 && kinds[k] != 1) return fail(TACCEL_ERR_ARG, "debug_barrier: kind must be 0 or 1");
  Dev dk(sizeof(int) * n), dx(sizeof(double) * 12 * n), dm(sizeof(double) * n), de(sizeof(double) * n),
      dg(sizeof(double) * 12 * n), dH(sizeof(double) * 144 * n), dHp(sizeof(double) * 144 * n), dt(sizeof(int) * n);
  if (!dk.p || !dx.p || !dm.p || !de.p || !dg.p || !dH.p || !dHp.p || !dt.p) return fail(TACCEL_ERR_OOM, "debug_barrier: hipMalloc");
  taccel_status st;
  if ((st = hip_status(hipMemcpy(dk.p, kinds, sizeof(int) * n, hipMemcpyHostToDevice), "H2D")) != TACCEL_OK) return st;
  if ((st = hip_status(hipMemcpy(dx.p, x, sizeof(double) * 12 * n, hipMemcpyHostToDevice), "H2D")) != TACCEL_OK) return st;
  if ((st = hip_status(hipMemcpy(dm.p, meps, sizeof(double) * n, hipMemcpyHostToDevice), "H2D")) != TACCEL_OK) return st;
  tc::launch_debug_barrier(n, dk.as<int>(), dx.as<double>(), dm.as<double>(), dhat, kappa, de.as<double>(),
                           dg.as<double>(), dH.as<double>(), dHp.as<double>(), dt.as<int>(), nullptr);
  if ((st = hip_status(hipDeviceSynchronize(), "debug_barrier kernel")) != TACCEL_OK) return st;
  if ((st = fetch(e, de, n)) != TACCEL_OK) return st;
  if ((st = fetch(g, dg, 12 * (size_t)n)) != TACCEL_OK) return st;
  if ((st = fetch(H, dH, 144 * (size_t)n)) != TACCEL_OK) return st;
  if ((st = fetch(Hp, dHp, 144 * (size_t)n)) != TACCEL_OK) return st;
  return fetch(types, dt, n);
}

taccel_status taccel_debug_friction(int32_t n, const int32_t* kinds, const double* xn, const double* x,
                                    const double* meps, double dhat, double kappa, double mu,
                                    double eps_v_h, double* lambda, double* e, double* g, double* H) {
  if (n < 0 || (n > 0 && (!kinds || !xn || !x || !meps || !lambda || !e || !g || !H)))
    return fail(TACCEL_ERR_ARG, "debug_friction: bad arguments");
  if (!(dhat > 0.0) || !(eps_v_h > 0.0) || !(mu >= 0.0))
    return fail(TACCEL_ERR_ARG, "debug_friction: dhat and eps_v_h must be > 0, mu >= 0");
  if (n == 0) return TACCEL_OK;
  for (int k = 0; k < n; ++k)
    if (kinds[k] != 0 && kinds[k] != 1) return fail(TACCEL_ERR_ARG, "debug_friction: kind must be 0 or 1");
  Dev dk(sizeof(int) * n), dxn(sizeof(double) * 12 * n), dx(sizeof(double) * 12 * n), dm(sizeof(double) * n),
      dl(sizeof(double) * n), de(sizeof(double) * n), dg(sizeof(double) * 12 * n), dH(sizeof(double) * 144 * n);
  if (!dk.p || !dxn.p || !dx.p || !dm.p || !dl.p || !de.p || !dg.p || !dH.p)
    return fail(TACCEL_ERR_OOM, "debug_friction: hipMalloc");
  taccel_status st;
  if ((st = hip_status(hipMemcpy(dk.p, kinds, sizeof(int) * n, hipMemcpyHostToDevice), "H2D")) != TACCEL_OK) return st;
  if ((st = hip_status(hipMemcpy(dxn.p, xn, sizeof(double) * 12 * n, hipMemcpyHostToDevice), "H2D")) != TACCEL_OK) return st;
  if ((st = hip_status(hipMemcpy(dx.p, x, sizeof(double) * 12 * n, hipMemcpyHostToDevice), "H2D")) != TACCEL_OK) return st;
  if ((st = hip_status(hipMemcpy(dm.p, meps, sizeof(double) * n, hipMemcpyHostToDevice), "H2D")) != TACCEL_OK) return st;
  tc::launch_debug_friction(n, dk.as<int>(), dxn.as<double>(), dx.as<double>(), dm.as<double>(), dhat, kappa, mu,
                            eps_v_h, dl.as<double>(), de.as<double>(), dg.as<double>(), dH.as<double>(), nullptr);
  if ((st = hip_status(hipDeviceSynchronize(), "debug_friction kernel")) != TACCEL_OK) return st;
  if ((st = fetch(lambda, dl, n)) != TACCEL_OK) return st;
  if ((st = fetch(e, de, n)) != TACCEL_OK) return st;
  if ((st = fetch(g, dg, 12 * (size_t)n)) != TACCEL_OK) return st;
  return fetch(H, dH, 144 * (size_t)n);
}

taccel_status taccel_debug_ccd(int32_t n, const int32_t* kinds, const double* x, const double* p,
                               double gap_ratio, int32_t max_iter, double* t) {
  if (n < 0 || (n > 0 && (!kinds || !x || !p || !t)) || max_iter <= 0 || !(gap_ratio > 0 && gap_ratio < 1))
    return fail(TACCEL_ERR_ARG, "debug_ccd: bad arguments");
  if (n == 0) return TACCEL_OK;
  for (int k = 0; k < n; ++k)
    if (kinds[k] != 0 && kinds[k] != 1) return fail(TACCEL_ERR_ARG, "debug_ccd: kind must be 0 or 1");
  Dev dk(sizeof(int) * n), dx(sizeof(double) * 12 * n), dp(sizeof(double) * 12 * n), dt(sizeof(double) * n);
  if (!dk.p || !dx.p || !dp.p || !dt.p) return fail(TACCEL_ERR_OOM, "debug_ccd: hipMalloc");
  taccel_status st;
  if ((st = hip_status(hipMemcpy(dk.p, kinds, sizeof(int) * n, hipMemcpyHostToDevice), "H2D")) != TACCEL_OK) return st;
  if ((st = hip_status(hipMemcpy(dx.p, x, sizeof(double) * 12 * n, hipMemcpyHostToDevice), "H2D")) != TACCEL_OK) return st;
  if ((st = hip_status(hipMemcpy(dp.p, p, sizeof(double) * 12 * n, hipMemcpyHostToDevice), "H2D")) != TACCEL_OK) return st;
  tc::launch_debug_ccd(n, dk.as<int>(), dx.as<double>(), dp.as<double>(), gap_ratio, max_iter, dt.as<double>(), nullptr);
  if ((st = hip_status(hipDeviceSynchronize(), "debug_ccd kernel")) != TACCEL_OK) return st;
  return fetch(t, dt, n);
}

taccel_status taccel_debug_arap(int32_t n, const double* A, double* e, double* g, double* H, double* Hp) {
  if (n < 0 || (n > 0 && !A)) return fail(TACCEL_ERR_ARG, "debug_arap: bad arguments");
  if (n == 0) return TACCEL_OK;
  Dev dA(sizeof(double) * 9 * n), de(sizeof(double) * n), dg(sizeof(double) * 9 * n), dH(sizeof(double) * 81 * n),
      dHp(sizeof(double) * 81 * n);
  if (!dA.p || !de.p || !dg.p || !dH.p || !dHp.p) return fail(TACCEL_ERR_OOM, "debug_arap: hipMalloc");
  taccel_status st;
  if ((st = hip_status(hipMemcpy(dA.p, A, sizeof(double) * 9 * n, hipMemcpyHostToDevice), "H2D")) != TACCEL_OK) return st;
  tc::launch_debug_arap(n, dA.as<double>(), de.as<double>(), dg.as<double>(), dH.as<double>(), dHp.as<double>(), nullptr);
  if ((st = hip_status(hipDeviceSynchronize(), "debug_arap kernel")) != TACCEL_OK) return st;
  if ((st = fetch(e, de, n)) != TACCEL_OK) return st;
  if ((st = fetch(g, dg, 9 * (size_t)n)) != TACCEL_OK) return st;
  if ((st = fetch(H, dH, 81 * (size_t)n)) != TACCEL_OK) return st;
  return fetch(Hp, dHp, 81 * (size_t)n);
}

void taccel_profile_enable(int32_t on) {
  tc::profiler().on = (on & 1) != 0;
  tc::profiler().phases = (on & 2) != 0;
}

void taccel_profile_reset(void) {
  tc::Profiler& p = tc::profiler();
  p.spmv_ms = 0.0;
  p.spmv_launches = 0;
  p.spmv_bytes = 0.0;
  p.pcg_ms = 0.0;
  p.pcg_iters = 0;
  p.refine_dirs = 0;
  p.refine_passes = 0;
  for (double& v : p.phase_ms) v = 0.0;
  p.phase_calls = 0;
}

taccel_status taccel_profile_query(const char* kernel, double* total_ms, int64_t* launches,
                                   double* algorithmic_bytes) {
  const tc::Profiler& p = tc::profiler();
  if (kernel && std::strcmp(kernel, "spmv") == 0) {
    if (total_ms) *total_ms = p.spmv_ms;
    if (launches) *launches = p.spmv_launches;
    if (algorithmic_bytes) *algorithmic_bytes = p.spmv_bytes;
    return TACCEL_OK;
  }
  if (kernel && std::strcmp(kernel, "pcg") == 0) {
    if (total_ms) *total_ms = p.pcg_ms;
    if (launches) *launches = p.pcg_iters;
    if (algorithmic_bytes) *algorithmic_bytes = 0.0;
    return TACCEL_OK;
  }
  if (kernel && std::strcmp(kernel, "refine") == 0) {
    // launches: FP32 passes; algorithmic_bytes: the Newton directions they solved
    if (total_ms) *total_ms = 0.0;
    if (launches) *launches = p.refine_passes;
    if (algorithmic_bytes) *algorithmic_bytes = (double)p.refine_dirs;
    return TACCEL_OK;
  }
  for (int k = 0; kernel && k < tc::Profiler::kPhases; ++k)
    if (std::strcmp(kernel, tc::kPhaseNames[k]) == 0) {
      if (total_ms) *total_ms = p.phase_ms[k];
      if (launches) *launches = p.phase_calls;
      if (algorithmic_bytes) *algorithmic_bytes = 0.0;
      return TACCEL_OK;
    }
  return fail(TACCEL_ERR_ARG, "profile_query: \"spmv\", \"pcg\", \"refine\" or a Newton-iteration phase name");
}

taccel_status taccel_device_synchronize(void) {
  return hip_status(hipDeviceSynchronize(), "hipDeviceSynchronize");
}

}  // extern "C"
