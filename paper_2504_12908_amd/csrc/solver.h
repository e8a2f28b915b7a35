// Internal interface of the batched IPC time-step solver (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/taccel.h"

namespace tc {

constexpr int kTrials = 8;        // line-search step sizes evaluated per launch
constexpr int kNodeChunk = 64;    // nodes per workgroup in node-parallel kernels (multiple of 4)
constexpr int kRowChunk = 16;     // block-rows per workgroup of the sparse product
constexpr int kTetChunk = 256;

// Per-scene constants, resident on the device.
struct SceneConst {
  double h, dhat, kappa, kappa_s, stop, mu, lam, pcg_eta;
  double fmu, eh;  // friction coefficient (0: none) and eps_v * h
  double grav[3];
  double cell, org[3];
  int node0, node1, tet0, tet1, cv0, cv1, q0, q1, body0, body1, tri0, tri1, edge0, edge1;
  int precision;
  int forcing;  // 1: PCG tolerance per Newton iteration by the forcing rule (pcg_forcing)
};

// Raw device pointers of a batch; passed by value to every kernel.
struct View {
  int S, Nn, Nt, Nb, Ncv, Ntr, Ned, Nq;
  const SceneConst* sc;
  // nodes: soft vertices, padding, 4 pseudo-nodes per affine body (p, c1, c2, c3)
  double *x, *xn, *xhat, *v;
  const double* xrest;  // creation (rest) positions
  const double* mass;
  int* nfree;        // 1 if the node's 3 dofs are unknowns
  const int* nscene;
  const int* nbody;  // body of a pseudo-node, -1 otherwise
  const int* ntype;  // 0 soft, 1 body p, 2 body c, 3 padding
  // tets (SoA)
  const int* tv;      // [4][Nt] node ids
  const double* Dminv;  // [9][Nt]
  const double* tvol;
  const int* tscene;
  // static BSR over nodes (FEM pattern)
  const int* rowptr;
  const int* col;
  double* val;
  const int* diag;
  const int* vptr;
  const int* vlist;  // tet*4 + a
  // bodies
  const int* bnode;
  const int* bscene;
  const double* bmass;  // m, Q[9]
  const double* bvol;
  const int* bpres;
  double* bstar;  // y* [12]
  double* blam;   // multipliers [12]
  double* bkap;   // penalty
  int* bsnap;
  double* bgrad;  // [12]
  double* bhess;  // [144]
  double* bpinv;  // [144]
  const int* bcv0;
  const int* bcv1;
  // contact vertices and primitives
  const int* cvn;
  const int* cvb;
  const double* cvx;  // xbar [3]
  const int* cvfix;
  const int* cvscene;
  const int* cvworld;
  double* cpos;
  double* cdisp;
  const int* trv;  // [Ntr][3] contact-vertex ids
  const int* edv;  // [Ned][2]
  const double* elen2;
  const int* qkind;  // 0: vertex (PT query), 1: edge (EE query)
  const int* qidx;
  const int* qscene;
  // per-scene state
  int* act;    // scene takes part in the current Newton iteration
  int* pdone;  // PCG finished for the scene
  // 1: the scene's FEM and barrier Hessians enter the Newton system exactly (unprojected) in
  // this iteration; 0: projected to positive semidefinite
  const int* exact;
};

// A batch of independent scenes solved together.
class Batch {
 public:
  static taccel_status create(const taccel_scene_desc* d, int n, const taccel_runtime* rt,
                              Batch** out, std::string& err);
  // host-side checks of create() only (no device call)
  static taccel_status validate(const taccel_scene_desc* d, int n, std::string& err);
  ~Batch();
  // mask (nullable): scenes with mask[k] == 0 are left untouched by this call
  taccel_status step(const taccel_targets* t, taccel_status* per_scene, taccel_step_stats* st,
                     const int* mask = nullptr);
  size_t device_bytes() const;  // device memory the object holds now
  // Device memory the object may hold from now on (0: no limit); an allocation past it fails
  // the call that needs it with TACCEL_ERR_OOM.
  void set_byte_limit(size_t bytes);
  taccel_status read(int scene, taccel_field f, void* dst, size_t bytes);
  taccel_status write(int scene, taccel_field f, const void* src, size_t bytes);
  taccel_status field_bytes(int scene, taccel_field f, size_t* bytes);
  taccel_status read_device(int scene, taccel_field f, void* dst, size_t bytes);
  // creation state for the scenes with mask[k] != 0 (all when mask is NULL)
  taccel_status reset(const uint8_t* mask);
  taccel_status debug_system(const taccel_targets* t, double* grad, int32_t* brow, int32_t* bcol,
                             double* bval, int32_t cap, int32_t* n_blocks);
  taccel_status debug_candidates(const double* P0, const double* P1, int32_t* out, int32_t cap,
                                 int32_t* n);
  taccel_status markers(int scene, int m, const int32_t* tris, const double* bary, double* pos,
                        double* flow);
  taccel_status depth_map(int scene, const taccel_camera* cam, int ntri, const int32_t* tris,
                          double* depth, double* normal);
  int num_scenes() const { return S_; }
  // Everything of scene k that carries from one step to the next (node positions and
  // velocities in the batch's internal order, the bodies' multipliers), bit for bit: a batch
  // built from the same scene description takes it with import_state and continues exactly as
  // this one would.
  struct SceneState {
    std::vector<double> x, v, lam;
  };
  taccel_status export_state(int scene, SceneState& out);
  taccel_status import_state(int scene, const SceneState& in);

  struct Impl;
  Impl* impl_ = nullptr;

 private:
  int S_ = 0;
};

void set_last_error(const std::string& msg);

}  // namespace tc
