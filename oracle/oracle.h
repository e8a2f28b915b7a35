/* CPU FP64 oracle of the unified ABD-IPC time step (Taccel, arXiv 2504.12908, Sec. 3 and
 * App. A).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that the GPU
 * library is checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no source with the GPU library.
 *
 * Every exported routine is a C function over plain host pointers.  Lengths are in metres,
 * SI units throughout.  Indices are 0-based int32.  Arrays marked [n][k] are row-major.
 */
#ifndef TACCEL_ORACLE_H
#define TACCEL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Scene description.  Soft body: nv vertices, nt positively oriented tets, dirichlet flag
 * per vertex (0 free, 1 fixed, 2 moving; NULL = all free).  Affine bodies: nb closed,
 * outward-oriented triangle meshes given by their creation-pose world vertices,
 * concatenated (body_nv / body_nf give the counts; body_tris indices are local to the
 * body). */
typedef struct {
  int32_t nv;
  const double* verts;        /* [nv][3] rest = initial positions */
  int32_t nt;
  const int32_t* tets;        /* [nt][4] */
  const uint8_t* dirichlet;   /* [nv] or NULL */
  double youngs, poisson, density;
  int32_t nb;
  const int32_t* body_nv;     /* [nb] */
  const int32_t* body_nf;     /* [nb] */
  const double* body_verts;   /* [sum nv][3] */
  const int32_t* body_tris;   /* [sum nf][3], local indices */
  const double* body_density; /* [nb] */
  const int32_t* body_prescribed; /* [nb] 1: kinematic target each step */
  double h, dhat, kappa, kappa_s, newton_tol;
  double gravity[3];
  int32_t max_newton, max_al;
  double friction; /* Coulomb coefficient mu of the lagged friction potential; 0: frictionless */
  double eps_v;    /* static/dynamic velocity threshold of the friction mollifier (m/s) */
} orc_desc;

typedef struct {
  int32_t status;        /* 0 ok, 3 not converged, 4 line search failed, 5 AL failed,
                            6 NaN, 7 infeasible target */
  int32_t newton_iters;  /* summed over all Newton loops of the step */
  int32_t al_rounds;     /* Newton loops run (1 + number of multiplier updates/snaps) */
} orc_stats;

void* orc_create(const orc_desc* d, char* err, int32_t errlen);
void orc_destroy(void* s);
/* body_targets: [nb][12] world affine maps of creation-pose vertices (t[3], A row-major[9]),
 * used for prescribed bodies; dir_targets: [n_moving][3] positions of the vertices flagged
 * 2, in increasing vertex order. */
int32_t orc_step(void* s, const double* body_targets, const double* dir_targets,
                 orc_stats* st);
/* The same step in two halves, so a test can inspect the system at the start of the step:
 * orc_step_begin predicts, sets the targets and the friction lag and moves the moving
 * Dirichlet vertices (returns 0 or 7); orc_step_finish runs the Newton loops and the
 * augmented-Lagrangian rounds and returns the status of orc_step. */
int32_t orc_step_begin(void* s, const double* body_targets, const double* dir_targets);
int32_t orc_step_finish(void* s, orc_stats* st);
/* Newton system of the current state, over the current unknowns: free soft vertices in
 * increasing order (one 3-dof node each), then 4 pseudo-nodes (p, c1, c2, c3) per affine body
 * not fixed on its target; the pairs closer than dhat at the current positions are active.
 * terms selects energy terms (1 inertia, 2 elasticity, 4 body orthogonality, 8 kinematic
 * constraint, 16 barrier, 32 friction; 63 all).  Writes the energy, the gradient
 * G[3 n_nodes] (at most g_cap values), the projected Hessian as 3x3 blocks (row node, column
 * node, 9 values row-major; at most blk_cap blocks; *n_blocks gets the count) and node_of
 * [nv + nb]: first node of each soft vertex and body, -1 when it has none.  Returns n_nodes. */
int32_t orc_system(const void* s, uint32_t terms, double* energy, double* G, int32_t g_cap,
                   int32_t* brow, int32_t* bcol, double* bval, int32_t blk_cap, int32_t* n_blocks,
                   int32_t* node_of);
/* Newton direction p = -H^-1 G of that system (all terms) by the skyline Cholesky solve.
 * Returns n_nodes, or -1 when the factorisation breaks down. */
int32_t orc_newton_direction(const void* s, double* p, int32_t cap);
int32_t orc_num_world_verts(const void* s);
double orc_scene_scale(const void* s); /* rest bounding-box diagonal of the whole scene */
/* Brute-force minimum distance over all admissible pairs, minimum det(F) over tets and the
 * number of pairs closer than dhat, at the current state. */
void orc_diagnostics(const void* s, double* min_distance, double* min_volume_ratio,
                     int32_t* n_active);
/* x,v: [nv][3]; q,qd: [nb][12] in the public (t, A row-major) convention. */
void orc_get_state(const void* s, double* x, double* v, double* q, double* qd);
void orc_set_state(void* s, const double* x, const double* v, const double* q,
                   const double* qd);
/* World positions of all contact-capable vertices: soft vertices, then body vertices. */
void orc_world_positions(const void* s, double* out);
/* Newton log of the last step: 8 values per Newton iteration (augmented-Lagrangian round
 * from 1, iteration within its loop, max vertex displacement of the direction, CCD bound,
 * accepted step size, active pairs, largest kappa_A and body residual over the prescribed
 * bodies not yet snapped, after the update).  Returns the number of values. */
int32_t orc_newton_log(const void* s, double* out, int32_t cap);
/* Line-search log of the last step: pairs (E(z), E(z+alpha p)) for each Newton update. */
int32_t orc_ls_log(const void* s, double* out, int32_t cap);

/* Broad phase by brute force on given world positions P0 (and P1 for the swept test, or
 * NULL).  Each candidate is written as 5 int32: kind (0 point-triangle, 1 edge-edge) and
 * four world vertex ids in canonical order (PT: point, sorted triangle; EE: sorted first
 * edge, sorted second edge, the lexicographically smaller edge first).  Returns the count
 * (writes at most cap). */
int32_t orc_candidates(const void* s, const double* P0, const double* P1, int32_t* out,
                       int32_t cap);

/* Pure evaluators (no scene). */
void orc_nh_tet(const double rest[12], const double x[12], double mu, double lam,
                double* e, double g[12], double H[144], double Hp[144]);
int32_t orc_pair_barrier(int32_t kind, const double x[12], double mollifier_eps,
                         double dhat, double kappa, double* e, double g[12],
                         double H[144], double Hp[144]);
double orc_pair_sqdist(int32_t kind, const double x[12], int32_t* dtype);
double orc_accd(int32_t kind, const double x[12], const double p[12], double gap_ratio,
                int32_t max_iter);
double orc_barrier(double d, double dhat, double* d1, double* d2);
void orc_abd_mass(int32_t nv, const double* verts, int32_t nf, const int32_t* tris,
                  double rho, double out[14]); /* m, volume, com[3], Q[9] */
double orc_arap(const double A[9], double g[9], double H[81], double Hp[81]);
/* Friction potential of one pair (App. A.3): the lagged data (closest-point weights, normal,
 * normal-force magnitude lambda) are taken at xn[12]; returns lambda and writes the energy
 * mu*lambda*f0(|u|) of the configuration x[12] and its gradient and Hessian (no h^2 factor). */
double orc_pair_friction(int32_t kind, const double xn[12], const double x[12], double mollifier_eps,
                         double dhat, double kappa, double mu, double eps_v_h, double* e,
                         double g[12], double H[144]);
void orc_psd_project(int32_t n, const double* A, double* out);

#ifdef __cplusplus
}
#endif
#endif
