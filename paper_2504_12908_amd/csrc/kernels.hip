// Kernels of the batched IPC time step (gfx950, wave64).
//
// Layout: node vectors are AoS [node][3] (gathers read 24 contiguous bytes); tet data is
// SoA ([k][Nt]) so consecutive threads read consecutive words.  Scenes are concatenated;
// node- and tet-parallel kernels that reduce use scene-aligned block tables so every
// partial sum belongs to one scene and per-scene reductions run in a fixed order
// (deterministic results, independent of what else is in the batch).
#include "contact.h"
#include "elastic.h"
#include "kernels.h"

namespace tc {
namespace {

constexpr int TPB = 256;
inline int nblk(int n, int t = TPB) { return n <= 0 ? 0 : (n + t - 1) / t; }
__device__ __forceinline__ int gid() { return blockIdx.x * blockDim.x + threadIdx.x; }

// Deterministic sum over a 256-thread workgroup (fixed butterfly + fixed wave order).
__device__ double block_sum256(double v, double* lds) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  const double r = (lds[0] + lds[1]) + (lds[2] + lds[3]);
  __syncthreads();
  return r;
}


__device__ __forceinline__ void atomic_max_pos(unsigned long long* a, double v) {
  atomicMax(a, (unsigned long long)__double_as_longlong(v));
}
__device__ __forceinline__ void atomic_min_pos(unsigned long long* a, double v) {
  atomicMin(a, (unsigned long long)__double_as_longlong(v));
}

// ------------------------------------------------------------------ predict & positions
__global__ void k_predict(View V) {
  const int n = gid();
  if (n >= V.Nn) return;
  const SceneConst& sc = V.sc[V.nscene[n]];
  const int type = V.ntype[n];
  const double h = sc.h;
  for (int c = 0; c < 3; ++c) {
    const double x = V.x[3 * n + c];
    V.xn[3 * n + c] = x;
    double xh = x;
    if (type == 0 || type == 1 || type == 2) xh = x + h * V.v[3 * n + c];
    if (type == 0 || (type == 1 && !V.bpres[V.nbody[n]])) xh += h * h * sc.grav[c];
    V.xhat[3 * n + c] = xh;
  }
}

__global__ void k_set_moving(double* x, int n, const int* nodes, const double* tgt) {
  const int k = gid();
  if (k >= n) return;
  for (int c = 0; c < 3; ++c) x[3 * nodes[k] + c] = tgt[3 * k + c];
}

__device__ __forceinline__ void body_point(const View& V, const double* y, int cv, double* out) {
  for (int c = 0; c < 3; ++c) {
    double acc = y[c];
    for (int j = 0; j < 3; ++j) acc += V.cvx[3 * cv + j] * y[3 + 3 * j + c];
    out[c] = acc;
  }
}

// World position (or displacement, for a node-space direction) of each contact vertex.
__global__ void k_cmap(View V, const double* src, double* out) {
  const int cv = gid();
  if (cv >= V.Ncv) return;
  const int n = V.cvn[cv];
  if (n >= 0) {
    for (int c = 0; c < 3; ++c) out[3 * cv + c] = src[3 * n + c];
  } else {
    const int n0 = V.bnode[V.cvb[cv]];
    body_point(V, src + 3 * n0, cv, out + 3 * cv);
  }
}

__global__ void k_cend(View V, double* cend) {
  const int k = gid();
  if (k >= 3 * V.Ncv) return;
  cend[k] = V.cpos[k] + V.cdisp[k];
}

// Displacement of the bodies flagged in cand from y to y* (everything else frozen).
__global__ void k_snap_disp(View V, const int* cand) {
  const int cv = gid();
  if (cv >= V.Ncv) return;
  const int b = V.cvb[cv];
  double d[3] = {0, 0, 0};
  if (b >= 0 && cand[b]) {
    double a[3], t[3];
    body_point(V, V.x + 3 * V.bnode[b], cv, a);
    body_point(V, V.bstar + 12 * b, cv, t);
    for (int c = 0; c < 3; ++c) d[c] = t[c] - a[c];
  }
  for (int c = 0; c < 3; ++c) V.cdisp[3 * cv + c] = d[c];
}

// Largest vertex distance between the current and the target pose of each body.
__global__ void k_body_resid(View V, unsigned long long* res) {
  const int cv = gid();
  if (cv >= V.Ncv) return;
  const int b = V.cvb[cv];
  if (b < 0 || !V.bpres[b]) return;
  double a[3], t[3];
  body_point(V, V.x + 3 * V.bnode[b], cv, a);
  body_point(V, V.bstar + 12 * b, cv, t);
  const double r = sqrt((a[0] - t[0]) * (a[0] - t[0]) + (a[1] - t[1]) * (a[1] - t[1]) +
                        (a[2] - t[2]) * (a[2] - t[2]));
  atomic_max_pos(res + b, r);
}

// ------------------------------------------------------------------ broad phase
__device__ __forceinline__ int cell_of(double v, double org, double inv) {
  // fmin/fmax map NaN to the bound, so the result is always a finite cell index
  const double c = fmax(-1048576.0, fmin(1048576.0, floor((v - org) * inv)));
  return (int)c;
}
// Bucket of (scene, cell, primitive type): triangles and edges of one cell land in different
// buckets so a point query never scans edges and an edge query never scans triangles.
__device__ __forceinline__ int bucket_of(int s, int cx, int cy, int cz, int type, int mask) {
  uint64_t h = (uint64_t)(uint32_t)(2 * s + type) * 0x9E3779B97F4A7C15ull;
  h ^= (uint64_t)(uint32_t)cx * 0xC2B2AE3D27D4EB4Full;
  h ^= (uint64_t)(uint32_t)cy * 0x165667B19E3779F9ull;
  h ^= (uint64_t)(uint32_t)cz * 0xD6E8FEB86659FD93ull;
  h ^= h >> 29;
  h *= 0xBF58476D1CE4E5B9ull;
  h ^= h >> 32;
  return (int)(h & (uint64_t)mask);
}
__device__ void prim_box(const double* P0, const double* P1, const int* ids, int n, double* lo,
                         double* hi) {
  for (int c = 0; c < 3; ++c) {
    lo[c] = INFINITY;
    hi[c] = -INFINITY;
  }
  for (int k = 0; k < n; ++k)
    for (int c = 0; c < 3; ++c) {
      const double a = P0[3 * ids[k] + c];
      lo[c] = fmin(lo[c], a);
      hi[c] = fmax(hi[c], a);
      if (P1) {
        const double b = P1[3 * ids[k] + c];
        lo[c] = fmin(lo[c], b);
        hi[c] = fmax(hi[c], b);
      }
    }
}
// Cell range of a box grown by dhat.  A box longer than kMaxSpan cells on an axis, or
// covering more than kMaxCells cells, only arises from exploded positions or a runaway
// Newton direction: it is collapsed to its first cell (keeping every loop and every entry
// count bounded) and its scene is flagged, so the host fails that scene instead of using an
// incomplete candidate set.
constexpr int kMaxSpan = 64;
constexpr int kMaxCells = 4096;
__device__ void cell_range(const SceneConst& sc, const double* lo, const double* hi, int* cl,
                           int* overflow_s) {
  const double inv = 1.0 / sc.cell;
  bool bad = false;
  long long cells = 1;
  for (int c = 0; c < 3; ++c) {
    cl[c] = cell_of(lo[c] - sc.dhat, sc.org[c], inv);
    cl[3 + c] = cell_of(hi[c] + sc.dhat, sc.org[c], inv);
    if (cl[3 + c] < cl[c]) cl[3 + c] = cl[c];
    const int span = cl[3 + c] - cl[c] + 1;
    bad = bad || span > kMaxSpan;
    cells *= span > kMaxSpan ? kMaxSpan : span;
  }
  if (bad || cells > kMaxCells) {
    for (int c = 0; c < 3; ++c) cl[3 + c] = cl[c];
    atomicOr(overflow_s, 1);
  }
}
__device__ __forceinline__ int target_ids(const View& V, int t, int* ids) {
  if (t < V.Ntr) {
    ids[0] = V.trv[3 * t];
    ids[1] = V.trv[3 * t + 1];
    ids[2] = V.trv[3 * t + 2];
    return 3;
  }
  const int e = t - V.Ntr;
  ids[0] = V.edv[2 * e];
  ids[1] = V.edv[2 * e + 1];
  return 2;
}

__global__ void k_bp_targets(View V, const double* P0, const double* P1, BroadPhase bp, int all) {
  const int t = gid();
  if (t >= bp.ntarget) return;
  int ids[3];
  const int n = target_ids(V, t, ids);
  const int s = V.cvscene[ids[0]];
  if (!all && !V.act[s]) {
    bp.tncell[t] = 0;
    return;
  }
  double lo[3], hi[3];
  prim_box(P0, P1, ids, n, lo, hi);
  int cl[6];
  cell_range(V.sc[s], lo, hi, cl, bp.overflow + s);
  for (int c = 0; c < 3; ++c) {
    bp.tbox[6 * t + c] = lo[c];
    bp.tbox[6 * t + 3 + c] = hi[c];
  }
  for (int k = 0; k < 6; ++k) bp.tcell[6 * t + k] = cl[k];
  int cnt = 1;
  for (int c = 0; c < 3; ++c) cnt *= cl[3 + c] - cl[c] + 1;
  bp.tncell[t] = cnt;
}

__global__ void k_bp_count(View V, BroadPhase bp) {
  const int t = gid();
  if (t >= bp.ntarget || bp.tncell[t] == 0) return;
  int ids[3];
  target_ids(V, t, ids);
  const int s = V.cvscene[ids[0]];
  const int* cl = bp.tcell + 6 * t;
  const int type = t < V.Ntr ? 0 : 1;
  for (int z = cl[2]; z <= cl[5]; ++z)
    for (int y = cl[1]; y <= cl[4]; ++y)
      for (int x = cl[0]; x <= cl[3]; ++x)
        atomicAdd(bp.bcount + bucket_of(s, x, y, z, type, bp.table_mask), 1);
}

__global__ void k_bp_fill(View V, BroadPhase bp) {
  const int t = gid();
  if (t >= bp.ntarget || bp.tncell[t] == 0) return;
  int ids[3];
  target_ids(V, t, ids);
  const int s = V.cvscene[ids[0]];
  const int* cl = bp.tcell + 6 * t;
  const int type = t < V.Ntr ? 0 : 1;
  BpEntry E;
  E.t = t;
  for (int c = 0; c < 3; ++c) {
    E.lo[c] = bp.tbox[6 * t + c];
    E.hi[c] = bp.tbox[6 * t + 3 + c];
  }
  const int nv = type == 0 ? 3 : 2;
  E.v[0] = ids[0];
  E.v[1] = ids[1];
  E.v[2] = nv == 3 ? ids[2] : -1;
  E.scene = s;
  int body = V.cvb[ids[0]], fixed = V.cvfix[ids[0]] ? 1 : 0;
  for (int k = 1; k < nv; ++k) {
    if (V.cvb[ids[k]] != body) body = -1;
    if (!V.cvfix[ids[k]]) fixed = 0;
  }
  E.body = body;
  E.fixed = fixed;
  E.pad[0] = E.pad[1] = 0;
  for (int z = cl[2]; z <= cl[5]; ++z)
    for (int y = cl[1]; y <= cl[4]; ++y)
      for (int x = cl[0]; x <= cl[3]; ++x) {
        const int b = bucket_of(s, x, y, z, type, bp.table_mask);
        const int pos = bp.bstart[b] + atomicAdd(bp.bfill + b, 1);
        E.cx = x;
        E.cy = y;
        E.cz = z;
        bp.entries[pos] = E;
      }
}

__device__ __forceinline__ bool boxes_close_lohi(const double* a, const double* lo,
                                                 const double* hi, double dhat) {
  for (int c = 0; c < 3; ++c)
    if (!(a[c] - dhat <= hi[c] && lo[c] - dhat <= a[3 + c])) return false;
  return true;
}

// One query primitive per group of 16 lanes.  The lanes take 16 of the query's cells at a time
// and fetch their buckets' entry ranges together; an inclusive scan of the entry counts over
// the group (DPP, one row = one group) flattens those entries, and the lanes then test 16
// entries at a time, each finding its cell from the scan.  So the dependent loads of a query
// are paid once per 16 cells and once per 16 entries rather than once per cell.  Count pass:
// matches per query.  Emit pass: matches compacted in lane order with a ballot (the same tests
// in the same order, so each query emits exactly its count); k_bp_sort_queries then sorts each
// query's segment by target so the candidate list has the canonical order.
constexpr int kQueryLanes = 16;
__device__ __forceinline__ int row16_scan_int(int x) {  // inclusive scan within each DPP row
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);  // row_shr:8
  return x;
}
__global__ void __launch_bounds__(TPB) k_bp_query(View V, const double* P0, const double* P1,
                                                  BroadPhase bp, int all, int emit, int* cand_q,
                                                  int* cand_t) {
  __shared__ int sh_incl[TPB], sh_e0[TPB], sh_cell[TPB];
  const int sub = threadIdx.x & (kQueryLanes - 1);
  const int gbase = (int)threadIdx.x - sub;  // first thread of this lane's group
  const int q = blockIdx.x * (TPB / kQueryLanes) + (int)(threadIdx.x / kQueryLanes);
  if (q >= V.Nq) return;  // whole 16-lane group leaves together
  const int s = V.qscene[q];
  if (!all && !V.act[s]) {
    if (!emit && sub == 0) bp.qcount[q] = 0;
    return;
  }
  const int kind = V.qkind[q], i = V.qidx[q];
  int qids[2];
  int nq;
  if (kind == 0) {
    qids[0] = i;
    nq = 1;
  } else {
    qids[0] = V.edv[2 * i];
    qids[1] = V.edv[2 * i + 1];
    nq = 2;
  }
  const SceneConst& sc = V.sc[s];
  double qb[6];
  prim_box(P0, P1, qids, nq, qb, qb + 3);
  int ql[6];
  cell_range(sc, qb, qb + 3, ql, bp.overflow + s);
  const int off = emit ? bp.qoff[q] : 0;
  int cnt = 0;  // matches of this lane (count pass) / of the group so far (emit pass)
  const int qb0 = V.cvb[qids[0]];
  // query side of the admissibility tests: an edge query lies in body qb0 only if both its
  // vertices do; it is fixed only if all its vertices are
  const bool qbody = kind == 0 || V.cvb[qids[1]] == qb0;
  const bool qfix = V.cvfix[qids[0]] && (kind == 0 || V.cvfix[qids[1]]);
  const double inv = 1.0 / sc.cell;
  const int gshift = (threadIdx.x & 63) & ~(kQueryLanes - 1);
  const unsigned long long lt = (1ull << (threadIdx.x & 63)) - 1ull;
  // the cell box has at most kMaxCells cells (cell_range collapses larger ones)
  const int nx = ql[3] - ql[0] + 1, ny = ql[4] - ql[1] + 1, nz = ql[5] - ql[2] + 1;
  const int ncell = nx * ny * nz;
  for (int c0 = 0; c0 < ncell; c0 += kQueryLanes) {  // uniform over the group
    const int c = c0 + sub;
    int e0 = 0, ne = 0;
    if (c < ncell) {
      const int x = ql[0] + c % nx, y = ql[1] + (c / nx) % ny, z = ql[2] + c / (nx * ny);
      const int b = bucket_of(s, x, y, z, kind, bp.table_mask);
      e0 = bp.bstart[b];
      ne = bp.bcount[b];
    }
    const int incl = row16_scan_int(ne);
    const int total = __shfl(incl, kQueryLanes - 1, kQueryLanes);
    sh_incl[threadIdx.x] = incl;
    sh_e0[threadIdx.x] = e0;
    sh_cell[threadIdx.x] = c;
    __builtin_amdgcn_wave_barrier();
    for (int t0 = 0; t0 < total; t0 += kQueryLanes) {  // uniform over the group
      const int t = t0 + sub;
      bool hit = false;
      int tgt = 0;
      if (t < total) {
        int j = 0;  // the lane whose cell holds flattened entry t
        while (sh_incl[gbase + j] <= t) ++j;
        const int before = j > 0 ? sh_incl[gbase + j - 1] : 0;
        const int e = sh_e0[gbase + j] + (t - before);
        const int cc = sh_cell[gbase + j];
        const int x = ql[0] + cc % nx, y = ql[1] + (cc / nx) % ny, z = ql[2] + cc / (nx * ny);
        const BpEntry& E = bp.entries[e];
        const int tt = E.t;
        // a bucket may also hold entries of other keys that hash to it: the entry must be of
        // the query's scene, cell and primitive type (triangle targets for a point, edges for
        // an edge), or its target index would be read as the wrong kind of primitive
        hit = E.cx == x && E.cy == y && E.cz == z && E.scene == s && (tt >= V.Ntr) == (kind == 1) &&
              !(kind == 1 && tt - V.Ntr <= i) &&
              max(ql[0], cell_of(E.lo[0] - sc.dhat, sc.org[0], inv)) == x &&
              max(ql[1], cell_of(E.lo[1] - sc.dhat, sc.org[1], inv)) == y &&
              max(ql[2], cell_of(E.lo[2] - sc.dhat, sc.org[2], inv)) == z &&
              boxes_close_lohi(qb, E.lo, E.hi, sc.dhat);
        if (hit) {
          // admissibility: same scene, no shared vertex, not inside one body, not all fixed
          if (kind == 0) {
            tgt = tt;
            const int v = qids[0];
            hit = E.scene == s && v != E.v[0] && v != E.v[1] && v != E.v[2] &&
                  !(qb0 >= 0 && E.body == qb0) && !(qfix && E.fixed);
          } else {
            tgt = tt - V.Ntr;
            hit = E.scene == s && qids[0] != E.v[0] && qids[0] != E.v[1] && qids[1] != E.v[0] &&
                  qids[1] != E.v[1] && !(qb0 >= 0 && qbody && E.body == qb0) && !(qfix && E.fixed);
          }
        }
      }
      if (!emit) {
        cnt += hit;
      } else {
        const unsigned long long m = __ballot(hit);
        const unsigned long long mine = (m >> gshift) & 0xFFFFull;
        if (hit) {
          const int pos = off + cnt + __popcll(m & lt & (0xFFFFull << gshift));
          cand_q[pos] = q;
          cand_t[pos] = tgt;
        }
        cnt += __popcll(mine);
      }
    }
    __builtin_amdgcn_wave_barrier();  // this round's LDS entries are read before the next round
  }
  if (!emit) {
    for (int o = kQueryLanes / 2; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, kQueryLanes);
    if (sub == 0) bp.qcount[q] = cnt;
  }
}

// Canonical order inside each query's segment: ascending target.  One group of 16 lanes per
// query places every candidate at its stable rank (targets smaller than it, plus equal ones
// before it), reading the emitted order from tmp_t and writing the sorted one to cand_t.
__global__ void __launch_bounds__(TPB) k_bp_sort_queries(View V, BroadPhase bp, const int* tmp_t,
                                                         int* cand_t) {
  const int sub = threadIdx.x & (kQueryLanes - 1);
  const int q = blockIdx.x * (TPB / kQueryLanes) + (int)(threadIdx.x / kQueryLanes);
  if (q >= V.Nq) return;
  const int off = bp.qoff[q], cnt = bp.qcount[q];
  for (int i = sub; i < cnt; i += kQueryLanes) {
    const int ti = tmp_t[off + i];
    int rank = 0;
    for (int j = 0; j < cnt; ++j) {
      const int tj = tmp_t[off + j];
      rank += (tj < ti) || (tj == ti && j < i);
    }
    cand_t[off + rank] = ti;
  }
}

// ------------------------------------------------------------------ narrow phase
__device__ __forceinline__ int cand_verts(const View& V, int q, int t, int* ids) {
  const int kind = V.qkind[q], i = V.qidx[q];
  if (kind == 0) {
    ids[0] = i;
    ids[1] = V.trv[3 * t];
    ids[2] = V.trv[3 * t + 1];
    ids[3] = V.trv[3 * t + 2];
  } else {
    ids[0] = V.edv[2 * i];
    ids[1] = V.edv[2 * i + 1];
    ids[2] = V.edv[2 * t];
    ids[3] = V.edv[2 * t + 1];
  }
  return kind;
}
__device__ __forceinline__ void gather12(const double* P, const int* ids, double* x12) {
  for (int v = 0; v < 4; ++v)
    for (int c = 0; c < 3; ++c) x12[3 * v + c] = P[3 * ids[v] + c];
}

// Flag scenes with a candidate pair at zero distance (not a feasible IPC state).
__global__ void k_touching(View V, int n, const int* cq, const int* ct, int* bad) {
  const int k = gid();
  if (k >= n) return;
  int ids[4];
  const int kind = cand_verts(V, cq[k], ct[k], ids);
  double x12[12];
  gather12(V.cpos, ids, x12);
  if (!(pair_sqdist(kind, x12, nullptr) > 0.0)) bad[V.qscene[cq[k]]] = 1;
}

__global__ void k_diff3(int n3, const double* a, const double* b, double* out) {
  const int k = gid();
  if (k < n3) out[k] = a[k] - b[k];
}

// Flag scenes with a tet of non-positive det F at positions x.
__global__ void k_tets_positive(View V, const double* x, int* bad) {
  const int t = gid();
  if (t >= V.Nt) return;
  double x12[12], Dm[9], F[9];
  for (int v = 0; v < 4; ++v) {
    const int node = V.tv[v * V.Nt + t];
    for (int c = 0; c < 3; ++c) x12[3 * v + c] = x[3 * node + c];
  }
  for (int k = 0; k < 9; ++k) Dm[k] = V.Dminv[k * V.Nt + t];
  deformation_gradient(x12, Dm, F);
  if (!(det3(F) > 0.0)) bad[V.tscene[t]] = 1;
}

__global__ void k_narrow(View V, int n, const int* cq, const int* ct, int* flag) {
  const int k = gid();
  if (k >= n) return;
  int ids[4];
  const int kind = cand_verts(V, cq[k], ct[k], ids);
  double x12[12];
  gather12(V.cpos, ids, x12);
  const int s = V.qscene[cq[k]];
  const double dhat = V.sc[s].dhat;
  flag[k] = V.act[s] && pair_sqdist(kind, x12, nullptr) < dhat * dhat ? 1 : 0;
}

__global__ void k_compact_pairs(View V, int n, const int* cq, const int* ct, const int* flag,
                                const int* pos, int* pkind, int* pv, double* pmeps, int* pscene) {
  const int k = gid();
  if (k >= n || !flag[k]) return;
  const int o = pos[k];
  int ids[4];
  const int kind = cand_verts(V, cq[k], ct[k], ids);
  pkind[o] = kind;
  for (int v = 0; v < 4; ++v) pv[4 * o + v] = ids[v];
  pmeps[o] = kind == 1 ? 1e-3 * V.elen2[V.qidx[cq[k]]] * V.elen2[ct[k]] : 0.0;
  pscene[o] = V.qscene[cq[k]];
}

// Active pairs as records of the caller's world vertex ids: kind, then PT: point and sorted
// triangle; EE: both edges sorted, the lexicographically smaller edge first.
__global__ void k_contact_records(View V, int n, const int* cq, const int* ct, const int* flag,
                                  const int* pos, int* out) {
  const int k = gid();
  if (k >= n || !flag[k]) return;
  int ids[4];
  const int kind = cand_verts(V, cq[k], ct[k], ids);
  int w[4];
  for (int v = 0; v < 4; ++v) w[v] = V.cvworld[ids[v]];
  if (kind == 0) {
    if (w[1] > w[2]) { const int t = w[1]; w[1] = w[2]; w[2] = t; }
    if (w[2] > w[3]) { const int t = w[2]; w[2] = w[3]; w[3] = t; }
    if (w[1] > w[2]) { const int t = w[1]; w[1] = w[2]; w[2] = t; }
  } else {
    if (w[0] > w[1]) { const int t = w[0]; w[0] = w[1]; w[1] = t; }
    if (w[2] > w[3]) { const int t = w[2]; w[2] = w[3]; w[3] = t; }
    if (w[2] < w[0] || (w[2] == w[0] && w[3] < w[1])) {
      int t = w[0]; w[0] = w[2]; w[2] = t;
      t = w[1]; w[1] = w[3]; w[3] = t;
    }
  }
  int* o = out + 5 * (size_t)pos[k];
  o[0] = kind;
  for (int v = 0; v < 4; ++v) o[1 + v] = w[v];
}

// Readout into caller device memory: out[i] = src[idx[i]] for 3-vectors, and affine-body
// states y = [p; c1; c2; c3] (p at the centre of mass com0) turned into the public map
// q = (t = p - A com0, A row-major) of creation-pose vertices (for rates the same linear map).
__global__ void k_gather3(int n, const int* idx, const double* src, double* out) {
  const int i = gid();
  if (i >= n) return;
  const int j = idx[i];
  for (int c = 0; c < 3; ++c) out[3 * (size_t)i + c] = src[3 * (size_t)j + c];
}
__global__ void k_body_public(int nb, const double* y, const double* com0, double* out) {
  const int b = gid();
  if (b >= nb) return;
  const double* yb = y + 12 * (size_t)b;
  double* q = out + 12 * (size_t)b;
  for (int i = 0; i < 3; ++i) {
    double acc = yb[i];
    for (int j = 0; j < 3; ++j) acc -= yb[3 + 3 * j + i] * com0[3 * b + j];
    q[i] = acc;
    for (int j = 0; j < 3; ++j) q[3 + 3 * i + j] = yb[3 + 3 * j + i];
  }
}

// ------------------------------------------------------------------ FEM (one block-row per 32 lanes)
// Static rows of the Newton system straight from the tets: for soft node n, every tet that
// contains it (as its vertex a) is evaluated by one lane, which forms the tet's gradient entry
// at a and the four 3x3 blocks (a, b) of its 12x12 Hessian (the analytic singular-value
// eigensystem of the neo-Hookean density, every mode or only those of positive eigenvalue,
// pulled back to vertex space); the row's lanes then sum them per stored block in the tets'
// fixed order, add the lumped mass on the diagonal and write the row of the BSR and the
// node's gradient (inertia plus elasticity).  Nothing per tet goes to memory.  T is the
// type of the Hessian arithmetic and of the stored blocks: FP64, or FP32 in mixed precision,
// where the gradient entry also comes in FP32 from the displacement gradient G = F - I
// (formed from FP64 displacement differences) and is summed in FP64.
constexpr int kFemRowLanes = 32, kFemRows = 4, kFemChunk = 24;

// Entries 3a..3a+2 of a 12-vector, by selects rather than a dynamic index (which would put
// the vector in scratch memory).
template <class T>
__device__ __forceinline__ void pick3(const T* w, int a, T* out) {
  for (int i = 0; i < 3; ++i)
    out[i] = a == 0 ? w[i] : (a == 1 ? w[3 + i] : (a == 2 ? w[6 + i] : w[9 + i]));
}

template <class T>
__device__ void fem_row_entry(const View& V, const SceneConst& sc, int t, int a, bool exact,
                              double* gw, T* hw) {
  double x12[12], Dm[9];
  for (int v = 0; v < 4; ++v) {
    const int node = V.tv[v * V.Nt + t];
    for (int c = 0; c < 3; ++c) x12[3 * v + c] = V.x[3 * node + c];
  }
  for (int k = 0; k < 9; ++k) Dm[k] = V.Dminv[k * V.Nt + t];
  const double vol = V.tvol[t];
  const double scale = sc.h * sc.h * vol;
  T F[9], Dmt[9];
  for (int k = 0; k < 9; ++k) Dmt[k] = (T)Dm[k];
  if constexpr (sizeof(T) == sizeof(double)) {
    double Fd[9], P[9], w[12];
    deformation_gradient(x12, Dm, Fd);
    nh_stress(Fd, sc.mu, sc.lam, P);
    pullback(P, Dm, scale, w);
    double wa[3];
    pick3(w, a, wa);
    for (int c = 0; c < 3; ++c) gw[c] = wa[c];
    for (int k = 0; k < 9; ++k) F[k] = Fd[k];
  } else {
    // displacement differences in FP64, then G = (D_s - D_m) D_m^{-1} in FP32
    double u[12];
    for (int v = 0; v < 4; ++v) {
      const int node = V.tv[v * V.Nt + t];
      for (int c = 0; c < 3; ++c) u[3 * v + c] = x12[3 * v + c] - V.xrest[3 * node + c];
    }
    float Du[9], G[9], P[9], w[12];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) Du[3 * i + k] = (float)(u[3 * (k + 1) + i] - u[i]);
    matmul3(Du, Dmt, G);
    nh_stress_disp(G, (float)sc.mu, (float)sc.lam, P);
    pullback(P, Dmt, (float)scale, w);
    float wa[3];
    pick3(w, a, wa);
    for (int c = 0; c < 3; ++c) gw[c] = (double)wa[c];
    for (int k = 0; k < 9; ++k) F[k] = G[k] + ((k % 4 == 0) ? 1.0f : 0.0f);
  }
  ModesT<T> m;
  nh_modes(F, (T)sc.mu, (T)sc.lam, m);
  T acc[36];
  for (int k = 0; k < 36; ++k) acc[k] = (T)0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const T lk = m.lam[k];
    if (exact ? !isfinite(lk) : !(lk > (T)0)) continue;
    T Q[9], w[12], wa[3];
    mode_matrix(m, k, Q);
    pullback(Q, Dmt, (T)1, w);
    pick3(w, a, wa);
    for (int i = 0; i < 3; ++i) {
      const T wi = lk * wa[i];
      for (int j = 0; j < 12; ++j) acc[12 * i + j] += wi * w[j];
    }
  }
  const T sc_t = (T)scale;
  for (int b = 0; b < 4; ++b)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) hw[9 * b + 3 * i + j] = sc_t * acc[12 * i + 3 * b + j];
}

template <class T>
__global__ void __launch_bounds__(kFemRowLanes * kFemRows) k_fem_rows(View V, double* g) {
  __shared__ T hrow[kFemRows][kFemChunk][36];
  __shared__ double grow[kFemRows][kFemChunk][3];
  __shared__ int tcol[kFemRows][kFemChunk][4];
  __shared__ int cnt_s[kFemRows];
  const int r = (int)threadIdx.x / kFemRowLanes, lane = (int)threadIdx.x % kFemRowLanes;
  const int n = (int)blockIdx.x * kFemRows + r;
  const bool on = n < V.Nn && V.act[V.nscene[n]];
  const bool soft = on && V.ntype[n] == 0;
  const int k0 = soft ? V.vptr[n] : 0, cnt = soft ? V.vptr[n + 1] - k0 : 0;
  const int rb0 = soft ? V.rowptr[n] : 0, nbk = soft ? V.rowptr[n + 1] - rb0 : 0;
  if (lane == 0) cnt_s[r] = cnt;
  __syncthreads();
  int cmax = 0;
  for (int i = 0; i < kFemRows; ++i) cmax = max(cmax, cnt_s[i]);
  const int nchunk = max(1, (cmax + kFemChunk - 1) / kFemChunk);
  const bool exact = soft && V.exact[V.nscene[n]] != 0;
  T* val = reinterpret_cast<T*>(V.val);
  double gacc = 0.0;
  for (int ch = 0; ch < nchunk; ++ch) {
    const int c0 = ch * kFemChunk;
    const int m = min(kFemChunk, cnt - c0);  // tets of this row in this chunk (may be <= 0)
    if (lane < m) {
      const int code = V.vlist[k0 + c0 + lane];
      const int t = code >> 2, a = code & 3;
      fem_row_entry<T>(V, V.sc[V.nscene[n]], t, a, exact, grow[r][lane], hrow[r][lane]);
      for (int b = 0; b < 4; ++b) tcol[r][lane][b] = V.tv[b * V.Nt + t];
    }
    __syncthreads();
    for (int e = lane; e < 9 * nbk; e += kFemRowLanes) {
      const int kk = rb0 + e / 9, i = e % 9;
      const int c = V.col[kk];
      T acc = (T)0;
      for (int l = 0; l < m; ++l)
        for (int b = 0; b < 4; ++b)
          if (tcol[r][l][b] == c) acc += hrow[r][l][9 * b + i];
      if (ch == 0) {
        if (c == n && i % 4 == 0) acc += (T)V.mass[n];
        val[9 * (size_t)kk + i] = acc;
      } else {
        val[9 * (size_t)kk + i] += acc;
      }
    }
    if (lane < 3)
      for (int l = 0; l < m; ++l) gacc += grow[r][l][lane];
    __syncthreads();
  }
  if (on && lane < 3) {
    double gv = 0.0;
    if (soft && V.nfree[n]) gv = V.mass[n] * (V.x[3 * n + lane] - V.xhat[3 * n + lane]) + gacc;
    g[3 * (size_t)n + lane] = gv;
  }
}

// ------------------------------------------------------------------ wave-parallel Jacobi
// Frobenius-nearest PSD projection of a symmetric N x N matrix (N even) held in LDS by one
// wavefront: cyclic Jacobi in round-robin (tournament) order, N/2 disjoint rotations per
// round applied to A and to the eigenvector matrix V, ping-pong buffers, until the
// off-diagonal mass is below 1e-30 of the total; then V max(w, 0) V^T.  Result in A[0].
template <int N>
__device__ __forceinline__ int tour_index(int pos, int r) {  // index at a tournament position
  return pos == 0 ? 0 : 1 + (pos - 1 + r) % (N - 1);
}
template <int N>
__device__ __forceinline__ int tour_pos(int idx, int r) {
  return idx == 0 ? 0 : 1 + ((idx - 1 - r) % (N - 1) + (N - 1)) % (N - 1);
}
template <int N>
__device__ void wave_psd(double (&A)[2][N * N], double (&Vm)[2][N * N], double* cs, double* sn) {
  constexpr int NN = N * N, H = N / 2;
  const int lane = threadIdx.x;
  // round-robin schedule: partner of index i in round r and the slot of that pair
  __shared__ signed char partner[N - 1][N], slot[N - 1][N];
  for (int e = lane; e < (N - 1) * N; e += 64) {
    const int r = e / N, i = e % N;
    const int pi = tour_pos<N>(i, r);
    partner[r][i] = (signed char)tour_index<N>(N - 1 - pi, r);
    slot[r][i] = (signed char)(pi < H ? pi : N - 1 - pi);
  }
  int cur = 0;
  for (int e = lane; e < NN; e += 64) Vm[0][e] = (e / N == e % N) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = lane; e < NN; e += 64) {
      const double a = A[cur][e];
      tot += a * a;
      if (e / N != e % N) off += a * a;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o, 64);
      tot += __shfl_xor(tot, o, 64);
    }
    if (off <= 1e-30 * tot) break;
    for (int r = 0; r < N - 1; ++r) {
      if (lane < H) {
        int p = tour_index<N>(lane, r), q = tour_index<N>(N - 1 - lane, r);
        if (p > q) { const int t = p; p = q; q = t; }
        const double apq = A[cur][N * p + q];
        double c = 1.0, sg = 0.0;
        if (apq != 0.0) {
          const double theta = (A[cur][N * q + q] - A[cur][N * p + p]) / (2.0 * apq);
          const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          sg = t * c;
        }
        cs[lane] = c;
        sn[lane] = sg;
      }
      __syncthreads();
      const int nxt = cur ^ 1;
      for (int e = lane; e < 2 * NN; e += 64) {
        const bool isV = e >= NN;
        const int ee = isV ? e - NN : e;
        const int i = ee / N, j = ee % N;
        // rotation acting on column j: J[j][j] = c; J[oj][j] = -s if j is the smaller index
        // of its pair, else +s
        const int oj = partner[r][j], kj = slot[r][j];
        const double jjj = cs[kj], joj = j < oj ? -sn[kj] : sn[kj];
        if (isV) {
          Vm[nxt][ee] = Vm[cur][N * i + j] * jjj + Vm[cur][N * i + oj] * joj;
        } else {
          const int oi = partner[r][i], ki = slot[r][i];
          const double jii = cs[ki], joi = i < oi ? -sn[ki] : sn[ki];
          const double a_ij = A[cur][N * i + j], a_ioj = A[cur][N * i + oj];
          const double a_oij = A[cur][N * oi + j], a_oioj = A[cur][N * oi + oj];
          A[nxt][ee] = jii * (a_ij * jjj + a_ioj * joj) + joi * (a_oij * jjj + a_oioj * joj);
        }
      }
      __syncthreads();
      cur = nxt;
    }
  }
  // rebuild with clamped eigenvalues: out_ij = sum_k V_ik max(w_k, 0) V_jk
  const int nxt = cur ^ 1;
  for (int e = lane; e < NN; e += 64) {
    const int i = e / N, j = e % N;
    double acc = 0.0;
    for (int k = 0; k < N; ++k) {
      const double w = A[cur][(N + 1) * k];
      if (w > 0.0) acc += Vm[cur][N * i + k] * w * Vm[cur][N * j + k];
    }
    A[nxt][e] = acc;
  }
  __syncthreads();
  if (nxt != 0)
    for (int e = lane; e < NN; e += 64) A[0][e] = A[nxt][e];
  __syncthreads();
}

// ------------------------------------------------------------------ barrier (1 wave per pair)
// A pair's energy depends on vertex differences only, so its 12x12 Hessian vanishes on the
// three translations and is Q^T M Q for the 9x9 M = Q H Q^T, where Q = C (x) I3 and the rows
// of C (3x4) are orthonormal and orthogonal to (1,1,1,1).  Projecting M (padded to 10x10 with
// a zero row/column so the tournament has an even size) gives the projection of H.
__constant__ double kContrast[3][4] = {
    {0.70710678118654752440, -0.70710678118654752440, 0.0, 0.0},
    {0.40824829046386301637, 0.40824829046386301637, -0.81649658092772603273, 0.0},
    {0.28867513459481288225, 0.28867513459481288225, 0.28867513459481288225, -0.86602540378443864676}};

struct WaveBarrierLds {
  BarrierCore core;  // shared scalars of the pair (one lane computes them)
  double H[144];     // 12x12 Hessian, row-major; projected in place by wave_barrier_project
  double M[2][100];  // reduced 10x10
  double V[2][100];
  double c[5], s[5];
  double g[12];
};

// All 64 lanes: derivatives of one pair into L.H / L.g (entries spread over lanes).
__device__ void wave_barrier_derivs(int kind, const double* x12, double meps, double dhat,
                                    double kappa, WaveBarrierLds& L, double* e_out, int* type_out) {
  const int lane = threadIdx.x;
  if (lane == 0) barrier_core(kind, x12, meps, dhat, kappa, L.core);
  __syncthreads();
  const BarrierCore& B = L.core;
  if (lane < 12) L.g[lane] = barrier_grad_entry(B, lane);
  for (int e = lane; e < 144; e += 64) L.H[e] = barrier_hess_entry(B, e / 12, e % 12);
  *e_out = B.e;
  *type_out = B.type;
  __syncthreads();
}

__device__ void wave_barrier_project(WaveBarrierLds& L) {
  const int lane = threadIdx.x;
  for (int e = lane; e < 100; e += 64) {
    const int i = e / 10, j = e % 10;
    double acc = 0.0;
    if (i < 9 && j < 9) {
      const int al = i / 3, a = i % 3, be = j / 3, c = j % 3;
      for (int v = 0; v < 4; ++v) {
        const double cv = kContrast[al][v];
        if (cv == 0.0) continue;
        for (int w = 0; w < 4; ++w) {
          const double cw = kContrast[be][w];
          if (cw == 0.0) continue;
          acc += cv * cw * L.H[12 * (3 * v + a) + 3 * w + c];
        }
      }
    }
    L.M[0][e] = acc;
  }
  __syncthreads();
  wave_psd<10>(L.M, L.V, L.c, L.s);
  for (int e = lane; e < 144; e += 64) {
    const int va = e / 12 / 3, a = (e / 12) % 3, vc = (e % 12) / 3, c = e % 3;
    double acc = 0.0;
    for (int al = 0; al < 3; ++al) {
      const double cv = kContrast[al][va];
      if (cv == 0.0) continue;
      for (int be = 0; be < 3; ++be) {
        const double cw = kContrast[be][vc];
        if (cw == 0.0) continue;
        acc += cv * cw * L.M[0][10 * (3 * al + a) + 3 * be + c];
      }
    }
    L.H[e] = acc;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(64) k_barrier_hess(View V, int np, const int* pkind,
                                                     const int* pv, const double* pmeps, double* pg,
                                                     double* ph) {
  __shared__ WaveBarrierLds L;
  const int k = blockIdx.x;
  if (k >= np) return;
  int ids[4];
  for (int v = 0; v < 4; ++v) ids[v] = pv[4 * k + v];
  const SceneConst& sc = V.sc[V.cvscene[ids[0]]];
  double x12[12], e;
  int type;
  gather12(V.cpos, ids, x12);
  wave_barrier_derivs(pkind[k], x12, pmeps[k], sc.dhat, sc.h * sc.h * sc.kappa, L, &e, &type);
  // one pair per workgroup: the flag is uniform, so the projection's barriers are too
  if (!V.exact[V.cvscene[ids[0]]]) wave_barrier_project(L);
  if (threadIdx.x < 12) pg[12 * (size_t)k + threadIdx.x] = L.g[threadIdx.x];
  for (int i = threadIdx.x; i < 144; i += 64) ph[144 * (size_t)k + i] = L.H[i];
}

// ------------------------------------------------------------------ friction
// Lagged data of the n compacted pairs (closer than dhat at the start-of-step positions in
// cpos); one thread per pair.
__global__ void k_fric_build(View V, int n, const int* pkind, const int* pv, const double* pmeps,
                             FricBufs F) {
  const int k = gid();
  if (k >= n) return;
  int ids[4];
  for (int v = 0; v < 4; ++v) ids[v] = pv[4 * k + v];
  const SceneConst& sc = V.sc[V.cvscene[ids[0]]];
  double x12[12], w[4];
  gather12(V.cpos, ids, x12);
  const int kind = pkind[k];
  int type;
  const double s = pair_sqdist(kind, x12, &type);
  closest_point_weights(kind, type, x12, w);
  d3 c = mk(0, 0, 0);
  for (int v = 0; v < 4; ++v) c = c + w[v] * ld(x12 + 3 * v);
  const double cn = sqrt(dot(c, c));
  const bool ok = s > 0.0 && s < sc.dhat * sc.dhat && cn > 0.0;
  for (int v = 0; v < 4; ++v) {
    F.v[4 * k + v] = ids[v];
    F.w[4 * k + v] = w[v];
  }
  st(F.c0 + 3 * k, c);
  st(F.nrm + 3 * k, ok ? (1.0 / cn) * c : mk(0, 0, 0));
  F.mul[k] = ok ? sc.fmu * normal_force(kind, x12, s, pmeps[k], sc.dhat, sc.kappa) : 0.0;
}

// Friction pairs appended to the contact pair arrays at off..off+n-1: vertex ids, gradient
// and Hessian (times h^2) at the current positions; zero for scenes not iterating.
__global__ void k_fric_derivs(View V, FricBufs F, int off, int* pv, double* pg, double* ph) {
  const int k = gid();
  if (k >= F.n) return;
  int ids[4];
  double w[4];
  for (int v = 0; v < 4; ++v) {
    ids[v] = F.v[4 * k + v];
    w[v] = F.w[4 * k + v];
    pv[4 * (size_t)(off + k) + v] = ids[v];
  }
  const int s = V.cvscene[ids[0]];
  const SceneConst& sc = V.sc[s];
  double* G = pg + 12 * (size_t)(off + k);
  double* H = ph + 144 * (size_t)(off + k);
  const double mul = V.act[s] ? sc.h * sc.h * F.mul[k] : 0.0;
  if (mul == 0.0) {
    for (int i = 0; i < 12; ++i) G[i] = 0.0;
    for (int i = 0; i < 144; ++i) H[i] = 0.0;
    return;
  }
  double x12[12];
  gather12(V.cpos, ids, x12);
  friction_derivs(x12, w, ld(F.c0 + 3 * k), ld(F.nrm + 3 * k), mul, sc.eh, G, H);
}

// ------------------------------------------------------------------ affine bodies
// Inertia 1/2 dy^T My dy with My = diag(m I3, Q (x) I3), y = [p; c1; c2; c3].
__device__ void my_apply(const double* bm, const double* dy, double* out) {
  for (int c = 0; c < 3; ++c) out[c] = bm[0] * dy[c];
  for (int j = 0; j < 3; ++j)
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += bm[1 + 3 * j + k] * dy[3 + 3 * k + c];
      out[3 + 3 * j + c] = acc;
    }
}
__device__ __forceinline__ double my_entry(const double* bm, int r, int c) {
  const int ur = r / 3, uc = c / 3;
  if ((r % 3) != (c % 3)) return 0.0;
  if (ur == 0 || uc == 0) return (ur == 0 && uc == 0) ? bm[0] : 0.0;
  return bm[1 + 3 * (ur - 1) + (uc - 1)];
}

__global__ void k_body_hess(View V) {
  const int b = gid();
  if (b >= V.Nb) return;
  const int s = V.bscene[b];
  if (!V.act[s] || V.bsnap[b]) return;
  const SceneConst& sc = V.sc[s];
  const int n0 = V.bnode[b];
  const double* y = V.x + 3 * n0;
  const double* yh = V.xhat + 3 * n0;
  const double* bm = V.bmass + 10 * b;
  double dy[12], g[12];
  for (int k = 0; k < 12; ++k) dy[k] = y[k] - yh[k];
  my_apply(bm, dy, g);
  double* H = V.bhess + 144 * b;
  for (int r = 0; r < 12; ++r)
    for (int c = 0; c < 12; ++c) H[12 * r + c] = my_entry(bm, r, c);
  double A[9], gA[9], e;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[3 * i + j] = y[3 + 3 * j + i];
  Modes m;
  arap_modes(A, m, &e, gA);
  const double ks = sc.h * sc.h * sc.kappa_s * V.bvol[b];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) g[3 + 3 * j + i] += ks * gA[3 * i + j];
  for (int k = 0; k < 9; ++k) {
    const double lk = m.lam[k];
    if (!(lk > 0.0)) continue;
    double Q[9];
    mode_matrix(m, k, Q);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        for (int ii = 0; ii < 3; ++ii)
          for (int jj = 0; jj < 3; ++jj)
            H[12 * (3 + 3 * j + i) + 3 + 3 * jj + ii] += ks * lk * Q[3 * i + j] * Q[3 * ii + jj];
  }
  if (V.bpres[b]) {
    const double kap = V.bkap[b];
    double c[12], mc[12], ml[12];
    for (int k = 0; k < 12; ++k) c[k] = y[k] - V.bstar[12 * b + k];
    my_apply(bm, c, mc);
    my_apply(bm, V.blam + 12 * b, ml);
    for (int k = 0; k < 12; ++k) g[k] += kap * mc[k] - ml[k];
    for (int r = 0; r < 12; ++r)
      for (int cc = 0; cc < 12; ++cc) H[12 * r + cc] += kap * my_entry(bm, r, cc);
  }
  for (int k = 0; k < 12; ++k) V.bgrad[12 * b + k] = g[k];
}

// ------------------------------------------------------------------ assembly
// Node entries (node, weight) through which a contact vertex moves.
__device__ __forceinline__ int vertex_nodes(const View& V, int cv, int* node, double* w) {
  const int n = V.cvn[cv];
  if (n >= 0) {
    if (!V.nfree[n]) return 0;
    node[0] = n;
    w[0] = 1.0;
    return 1;
  }
  const int b = V.cvb[cv];
  if (V.bsnap[b]) return 0;
  const int n0 = V.bnode[b];
  node[0] = n0;
  w[0] = 1.0;
  for (int j = 0; j < 3; ++j) {
    node[1 + j] = n0 + 1 + j;
    w[1 + j] = V.cvx[3 * cv + j];
  }
  return 4;
}

__global__ void k_contrib_count(View V, int np, const int* pv, int* hcnt, int* gcnt) {
  const int k = gid();
  if (k >= np + V.Nb) return;
  int tot = 0;
  if (k < np) {
    int node[4];
    double w[4];
    for (int a = 0; a < 4; ++a) tot += vertex_nodes(V, pv[4 * k + a], node, w);
  } else {
    const int b = k - np;
    if (V.act[V.bscene[b]] && !V.bsnap[b]) tot = 4;
  }
  hcnt[k] = tot * tot;
  gcnt[k] = tot;
}

// Contribution source codes: >= 0 pair block/vector, < 0 body block/vector (-1 - code).
__global__ void k_contrib_emit(View V, int np, const int* pv, const int* hoff, const int* goff,
                               uint64_t* hkey, int* hidx, int* hsrc, double* hcoef, uint64_t* gkey,
                               int* gidx, int* gsrc, double* gcoef) {
  const int k = gid();
  if (k >= np + V.Nb) return;
  const uint64_t Nn = (uint64_t)V.Nn;
  int ho = hoff[k], go = goff[k];
  if (k < np) {
    int node[4][4], cnt[4];
    double w[4][4];
    for (int a = 0; a < 4; ++a) cnt[a] = vertex_nodes(V, pv[4 * k + a], node[a], w[a]);
    for (int a = 0; a < 4; ++a)
      for (int ia = 0; ia < cnt[a]; ++ia) {
        gkey[go] = (uint64_t)node[a][ia];
        gidx[go] = go;
        gsrc[go] = 4 * k + a;
        gcoef[go] = w[a][ia];
        ++go;
        for (int b = 0; b < 4; ++b)
          for (int ib = 0; ib < cnt[b]; ++ib) {
            hkey[ho] = (uint64_t)node[a][ia] * Nn + (uint64_t)node[b][ib];
            hidx[ho] = ho;
            hsrc[ho] = 16 * k + 4 * a + b;
            hcoef[ho] = w[a][ia] * w[b][ib];
            ++ho;
          }
      }
  } else {
    const int b = k - np;
    if (!V.act[V.bscene[b]] || V.bsnap[b]) return;
    const int n0 = V.bnode[b];
    for (int u = 0; u < 4; ++u) {
      gkey[go] = (uint64_t)(n0 + u);
      gidx[go] = go;
      gsrc[go] = -1 - (4 * b + u);
      gcoef[go] = 1.0;
      ++go;
      for (int w = 0; w < 4; ++w) {
        hkey[ho] = (uint64_t)(n0 + u) * Nn + (uint64_t)(n0 + w);
        hidx[ho] = ho;
        hsrc[ho] = -1 - (16 * b + 4 * u + w);
        hcoef[ho] = 1.0;
        ++ho;
      }
    }
  }
}

__global__ void k_seg_flags(int n, const uint64_t* keys, int* flags) {
  const int i = gid();
  if (i >= n) return;
  flags[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}
__global__ void k_seg_start(int n, const int* flags, const int* segid, int* segstart) {
  const int i = gid();
  if (i >= n) return;
  if (flags[i]) segstart[segid[i]] = i;
  if (i == n - 1) segstart[segid[i] + flags[i]] = n;
}

template <class T>
__global__ void k_reduce_blocks(View V, int nmax, const int* nseg, const uint64_t* keys, const int* idx,
                                const int* segstart, const int* src, const double* coef,
                                const double* ph, int* drow, int* dcol, T* dval, int* rowcnt) {
  const int k = gid();
  if (k >= nmax || k >= *nseg) return;
  const int i0 = segstart[k], i1 = segstart[k + 1];
  const uint64_t key = keys[i0];
  const int row = (int)(key / (uint64_t)V.Nn), col = (int)(key % (uint64_t)V.Nn);
  T acc[9];
  for (int i = 0; i < 9; ++i) acc[i] = (T)0;
  for (int i = i0; i < i1; ++i) {
    const int c = idx[i];
    const int code = src[c];
    const double w = coef[c];
    const double* M;
    int a, b;
    if (code >= 0) {
      M = ph + 144 * (size_t)(code >> 4);
      a = (code >> 2) & 3;
      b = code & 3;
    } else {
      const int cc = -1 - code;
      M = V.bhess + 144 * (size_t)(cc >> 4);
      a = (cc >> 2) & 3;
      b = cc & 3;
    }
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) acc[3 * r + q] += (T)(w * M[12 * (3 * a + r) + 3 * b + q]);
  }
  drow[k] = row;
  dcol[k] = col;
  for (int i = 0; i < 9; ++i) dval[9 * (size_t)k + i] = acc[i];
  atomicAdd(rowcnt + row, 1);
}

__global__ void k_reduce_grad(View V, int nmax, const int* nseg, const uint64_t* keys, const int* idx,
                              const int* segstart, const int* src, const double* coef,
                              const double* pg, double* g) {
  const int k = gid();
  if (k >= nmax || k >= *nseg) return;
  const int i0 = segstart[k], i1 = segstart[k + 1];
  const int node = (int)keys[i0];
  double acc[3] = {0, 0, 0};
  for (int i = i0; i < i1; ++i) {
    const int c = idx[i];
    const int code = src[c];
    const double w = coef[c];
    const double* v = code >= 0 ? pg + 12 * (size_t)(code >> 2) + 3 * (code & 3)
                                : V.bgrad + 12 * (size_t)((-1 - code) >> 2) + 3 * ((-1 - code) & 3);
    for (int q = 0; q < 3; ++q) acc[q] += w * v[q];
  }
  for (int q = 0; q < 3; ++q) g[3 * node + q] += acc[q];
}

template <class T>
__global__ void k_precond_soft(View V, const int* drowptr, const int* dcol, const T* dval,
                               T* pinv, int* bad) {
  const int n = gid();
  if (n >= V.Nn) return;
  const int s = V.nscene[n];
  if (!V.act[s]) return;
  T* out = pinv + 9 * (size_t)n;
  if (V.ntype[n] != 0 || !V.nfree[n]) {
    for (int i = 0; i < 9; ++i) out[i] = (T)0;
    return;
  }
  double D[9];
  const T* sd = reinterpret_cast<const T*>(V.val) + 9 * (size_t)V.diag[n];
  for (int i = 0; i < 9; ++i) D[i] = (double)sd[i];
  for (int k = drowptr[n]; k < drowptr[n + 1]; ++k)
    if (dcol[k] == n)
      for (int i = 0; i < 9; ++i) D[i] += (double)dval[9 * (size_t)k + i];
  double C[9];
  cofactor3(D, C);
  const double det = D[0] * C[0] + D[1] * C[1] + D[2] * C[2];
  if (!(det > 0.0) || !isfinite(det)) {
    bad[s] = 1;
    for (int i = 0; i < 9; ++i) out[i] = (T)0;
    return;
  }
  // D symmetric: inverse = C^T / det = C / det
  for (int i = 0; i < 9; ++i) out[i] = (T)(C[i] / det);
}

// Inverse of the 12x12 block of an affine body (its 4 pseudo-nodes) by one wavefront:
// Gauss-Jordan with partial pivoting on [M | I] held in LDS.
template <class T>
__global__ void __launch_bounds__(64) k_precond_body(View V, const int* drowptr, const int* dcol,
                                                     const T* dval, int* bad) {
  __shared__ double M[12][24];
  __shared__ double f[12];
  __shared__ int piv_s;
  const int b = blockIdx.x;
  const int s = V.bscene[b];
  if (!V.act[s] || V.bsnap[b]) return;
  const int lane = threadIdx.x;
  const int n0 = V.bnode[b];
  for (int e = lane; e < 288; e += 64) M[e / 24][e % 24] = (e % 24 >= 12 && e % 24 - 12 == e / 24) ? 1.0 : 0.0;
  __syncthreads();
  if (lane < 4) {
    const int u = lane;
    for (int k = drowptr[n0 + u]; k < drowptr[n0 + u + 1]; ++k) {
      const int w = dcol[k] - n0;
      if (w < 0 || w > 3) continue;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[3 * u + i][3 * w + j] = (double)dval[9 * (size_t)k + 3 * i + j];
    }
  }
  __syncthreads();
  for (int c = 0; c < 12; ++c) {
    if (lane == 0) {
      int p = c;
      for (int r = c + 1; r < 12; ++r)
        if (fabs(M[r][c]) > fabs(M[p][c])) p = r;
      piv_s = p;
    }
    __syncthreads();
    const int p = piv_s;
    if (!(fabs(M[p][c]) > 0.0)) {
      if (lane == 0) bad[s] = 1;
      return;
    }
    if (p != c && lane < 24) {
      const double t = M[c][lane];
      M[c][lane] = M[p][lane];
      M[p][lane] = t;
    }
    __syncthreads();
    const double inv = 1.0 / M[c][c];
    __syncthreads();
    if (lane < 24) M[c][lane] *= inv;
    if (lane < 12) f[lane] = M[lane][c];
    __syncthreads();
    for (int e = lane; e < 288; e += 64) {
      const int r = e / 24, k = e % 24;
      if (r != c) M[r][k] -= f[r] * M[c][k];
    }
    __syncthreads();
  }
  T* bpinv = reinterpret_cast<T*>(V.bpinv);
  for (int e = lane; e < 144; e += 64) bpinv[144 * (size_t)b + e] = (T)M[e / 12][12 + e % 12];
}

// ------------------------------------------------------------------ PCG
// z = M^{-1} r for the node n (local index li inside the block; rs stages r in LDS).
template <class T>
__device__ __forceinline__ void precond_apply(const View& V, const T* pinv, int n, int n0blk,
                                              const T (*rs)[3], T* z) {
  // rs: r of the nodes of this block (a body's 4 pseudo-nodes never straddle blocks)
  const int type = V.ntype[n];
  if (!V.nfree[n]) {
    z[0] = z[1] = z[2] = (T)0;
    return;
  }
  if (type == 0) {
    const T* P = pinv + 9 * (size_t)n;
    const int li = n - n0blk;
    for (int i = 0; i < 3; ++i) z[i] = P[3 * i] * rs[li][0] + P[3 * i + 1] * rs[li][1] + P[3 * i + 2] * rs[li][2];
    return;
  }
  const int b = V.nbody[n];
  const int u = n - V.bnode[b];
  const int l0 = V.bnode[b] - n0blk;
  const T* P = reinterpret_cast<const T*>(V.bpinv) + 144 * b;
  for (int i = 0; i < 3; ++i) {
    T acc = (T)0;
    for (int w = 0; w < 4; ++w)
      for (int j = 0; j < 3; ++j) acc += P[12 * (3 * u + i) + 3 * w + j] * rs[l0 + w][j];
    z[i] = acc;
  }
}

// Node-parallel PCG kernels run one wavefront (64 nodes) per block of the table T; the
// sparse product runs 16 lanes per block-row over the table TS (16 rows per block).
// Workgroups are dealt to the 8 XCDs round-robin in launch order; the PCG kernels remap the
// launch index so that each XCD takes one contiguous run of table blocks (with the Morton
// node order, a compact part of the mesh whose vector entries stay in that XCD's L2).
constexpr int kXcds = 8;
__host__ __device__ __forceinline__ int xcd_grid(int nblk) { return (nblk + kXcds - 1) / kXcds * kXcds; }
__device__ __forceinline__ int xcd_block(int nblk) {
  const int per = (nblk + kXcds - 1) / kXcds;
  const int logical = ((int)blockIdx.x % kXcds) * per + (int)blockIdx.x / kXcds;
  return logical < nblk ? logical : -1;
}
constexpr int kWave = 64;
constexpr int kRowLanes = 16;

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
// N independent wavefront sums, interleaved so their shuffles overlap.
template <class T, int N>
__device__ __forceinline__ void wave_sum_n(T (&v)[N]) {
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += __shfl_xor(v[k], off, 64);
}
// Wavefront totals by DPP lane moves (VALU only, no LDS crossbar traffic), for code where all
// 64 lanes are active: an inclusive scan within each row of 16 lanes (shifts by 1, 2, 4, 8),
// then the row totals carried across rows (row broadcasts of lanes 15 and 31), so lane 63
// ends with the total, which every lane then reads.  The order of the additions is fixed.
template <int Ctrl, int RowMask, int BankMask, bool Bound>
__device__ __forceinline__ double dpp_move(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u & 0xffffffffull), Ctrl, RowMask, BankMask, Bound);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), Ctrl, RowMask, BankMask, Bound);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int Ctrl, int RowMask, int BankMask, bool Bound>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), Ctrl, RowMask, BankMask, Bound));
}
__device__ __forceinline__ double lane63(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), 63);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ float lane63(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
template <class T>
__device__ __forceinline__ T wave_total(T x) {
  x += dpp_move<0x111, 0xf, 0xf, true>(x);   // row_shr:1
  x += dpp_move<0x112, 0xf, 0xf, true>(x);   // row_shr:2
  x += dpp_move<0x114, 0xf, 0xf, true>(x);   // row_shr:4
  x += dpp_move<0x118, 0xf, 0xf, true>(x);   // row_shr:8
  x += dpp_move<0x142, 0xa, 0xf, false>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_move<0x143, 0xc, 0xf, false>(x);  // row_bcast:31 into rows 2 and 3
  return lane63(x);
}
// Sum over each row of 16 lanes (an inclusive DPP scan within the row): the total is valid
// in the row's last lane (lane & 15 == 15).  All lanes of the wave must be active.
template <class T>
__device__ __forceinline__ T row16_total(T x) {
  x += dpp_move<0x111, 0xf, 0xf, true>(x);  // row_shr:1
  x += dpp_move<0x112, 0xf, 0xf, true>(x);  // row_shr:2
  x += dpp_move<0x114, 0xf, 0xf, true>(x);  // row_shr:4
  x += dpp_move<0x118, 0xf, 0xf, true>(x);  // row_shr:8
  return x;
}
template <class T, int N>
__device__ __forceinline__ void wave_total_n(T (&v)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_total(v[k]);
}
// N sums over a 256-thread workgroup by DPP wavefront totals; lds holds 4 x N values.
template <class T, int N>
__device__ void block_total256_n(T (&v)[N], T* lds) {
  wave_total_n(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
    for (int k = 0; k < N; ++k) lds[N * wid + k] = v[k];
  __syncthreads();
  for (int k = 0; k < N; ++k) v[k] = (lds[k] + lds[N + k]) + (lds[2 * N + k] + lds[3 * N + k]);
  __syncthreads();
}

// Lane-strided partial sums of N arrays at once: acc[n] = P[n][b0[n] + lane] +
// P[n][b0[n] + lane + 64] + ... (entries below b1[n]), added in that order.  Each pass has
// U loads per array in flight, and every array's loads are issued before any of them is
// waited for, so N sums cost one memory round trip per pass rather than N.  An array with a
// shorter range contributes exact zeros past its end, so the result does not depend on U.
template <int U, int N, class T>
__device__ __forceinline__ void strided_sums(const T* const (&P)[N], const int (&b0)[N], const int (&b1)[N],
                                             int lane, T (&acc)[N]) {
  int len = 0;
#pragma unroll
  for (int n = 0; n < N; ++n) {
    acc[n] = (T)0;
    len = max(len, b1[n] - b0[n]);
  }
  for (int i0 = lane; i0 < len; i0 += kWave * U) {
    T v[N][U];
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = b0[n] + i0 + kWave * u;
        v[n][u] = k < b1[n] ? P[n][k] : (T)0;
      }
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
      for (int u = 0; u < U; ++u) acc[n] += v[n][u];
  }
}

// Block partials of r.z and, with the coarse level on, the restriction of the
// residual onto the rigid modes u = t + w x d of the block's aggregate (d = scaled rest offset
// from the aggregate centroid): P^T r = (sum r, sum d x r) over the block's soft nodes.  One
// wave per 64-node block; lane 0 returns the sums.
template <class T>
__device__ __forceinline__ void block_partials(const View& V, const PcgBufsT<T>& B, int blk, int n, bool live,
                                               const T* r, const T* z, T& rz) {
  T v[7] = {r[0] * z[0] + r[1] * z[1] + r[2] * z[2], (T)0, (T)0, (T)0, (T)0, (T)0, (T)0};
  if (B.cg_on) {
    if (live && V.ntype[n] == 0) {
      const T* d = B.cg_d + 3 * n;
      v[1] = r[0];
      v[2] = r[1];
      v[3] = r[2];
      v[4] = d[1] * r[2] - d[2] * r[1];
      v[5] = d[2] * r[0] - d[0] * r[2];
      v[6] = d[0] * r[1] - d[1] * r[0];
    }
    wave_total_n(v);
    if (threadIdx.x == 0)
      for (int k = 0; k < 6; ++k) B.cg_rc[6 * blk + k] = v[1 + k];
  } else {
    v[0] = wave_total(v[0]);
  }
  rz = v[0];
}

// Preconditioned CG with two kernels per iteration k (parity = k & 1):
//   k_pcg_dir_spmv: convergence test on |r_k|; beta_k = rz_k / rz_{k-1};
//                   p_k = z_k + beta_k p_{k-1} (written to the other p buffer) and
//                   q_k = A p_k with p_k formed on the fly from z and p_{k-1};
//   k_pcg_update:   alpha_k = rz_k / (p_k . q_k); x += alpha p; r -= alpha q; z = M^{-1} r.
// p_{-1} = 0 and rz_{-1} = 1 make iteration 0 start with p_0 = z_0.
// With the coarse level on, M^{-1} = D^{-1} + P A_c^{-1} P^T (additive two-level).  The
// restricted residual r_c = P^T r follows the same recurrence as r: the sparse product also
// restricts q_k (block partials), and k_pcg_update forms r_c,k+1 = r_c,k - alpha_k P^T q_k for
// the whole scene, solves the coarse system for its aggregate (e = rows of A_c^{-1} times
// r_c,k+1) and adds P e to z and r_c . e to the block partials of r.z, so one kernel boundary
// per half-iteration suffices.  At the start, k_pcg_init restricts r_0 directly and
// k_pcg_coarse applies the coarse correction to z_0.
template <class T>
__global__ void __launch_bounds__(kWave) k_pcg_init(View V, BlockTable TN, PcgBufsT<T> B) {
  const int blk = xcd_block(TN.nblk);
  if (blk < 0) return;
  __shared__ T rs[kWave][3];
  const int s = TN.sc[blk];
  if (V.pdone[s]) return;
  const int n0 = TN.b0[blk], n1 = TN.b1[blk];
  const int n = n0 + threadIdx.x;
  const bool live = n < n1;
  T r[3] = {(T)0, (T)0, (T)0};
  if (live) {
    const bool f = V.nfree[n];
    for (int c = 0; c < 3; ++c) {
      r[c] = f ? (T)(-B.g[3 * n + c]) : (T)0;
      B.r[3 * n + c] = r[c];
      B.dx[3 * n + c] = 0.0;
      B.p0[3 * n + c] = (T)0;
    }
  }
  for (int c = 0; c < 3; ++c) rs[threadIdx.x][c] = r[c];
  __syncthreads();
  T z[3] = {(T)0, (T)0, (T)0};
  if (live) {
    precond_apply<T>(V, B.pinv, n, n0, rs, z);
    for (int c = 0; c < 3; ++c) B.z[3 * n + c] = z[c];
  }
  T rz;
  block_partials<T>(V, B, blk, n, live, r, z, rz);
  if (threadIdx.x == 0) {
    B.P_rz0[blk] = rz;
    B.P_rz1[blk] = (T)1;
    if (!B.keep_gg) B.P_gg[blk] = rz;  // g^T D^{-1} g: the reference of the stopping test
  }
}

// One 3x3 block of the sparse product with its operands: the block, and z and p_{k-1} at its
// column.  None of it depends on beta, so it can be loaded before the scene scalars are known.
template <class T>
struct SpmvEntry {
  T a[9], z[3], p[3];
};
template <class T>
__device__ __forceinline__ void spmv_load(const T* val, const int* col, const T* z, const T* pold, int k,
                                          SpmvEntry<T>& e) {
  const T* A = val + 9 * (size_t)k;
  for (int i = 0; i < 9; ++i) e.a[i] = A[i];
  const int c = col[k];
  for (int i = 0; i < 3; ++i) {
    e.z[i] = z[3 * c + i];
    e.p[i] = pold[3 * c + i];
  }
}
// q += A (z + beta p_{k-1}) at the block's column
template <class T>
__device__ __forceinline__ void spmv_acc(const SpmvEntry<T>& e, T beta, T& q0, T& q1, T& q2) {
  const T p0 = e.z[0] + beta * e.p[0];
  const T p1 = e.z[1] + beta * e.p[1];
  const T p2 = e.z[2] + beta * e.p[2];
  q0 += e.a[0] * p0 + e.a[1] * p1 + e.a[2] * p2;
  q1 += e.a[3] * p0 + e.a[4] * p1 + e.a[5] * p2;
  q2 += e.a[6] * p0 + e.a[7] * p1 + e.a[8] * p2;
}

// One wave covers 4 block-rows (16 lanes each); every wave computes the scene scalars
// itself, so the row loads are not held back behind a workgroup barrier (the only barrier
// is in the closing p.q reduction).  Each lane's first block of the static range (for most
// rows every block: a row of the tet mesh has at most 15 static blocks) is loaded, operands
// included, before the scene scalars, so the two chains of dependent loads overlap instead
// of following each other.  The dynamic (contact and body) blocks, present on few rows,
// follow the scalars: prefetching them too would cost occupancy on every row.
template <class T>
__global__ void __launch_bounds__(TPB) k_pcg_dir_spmv(View V, BlockTable TN, BlockTable TS, PcgBufsT<T> B,
                                                      int parity) {
  const int blk = xcd_block(TS.nblk);
  if (blk < 0) return;
  const int s = TS.sc[blk];
  // The blocks of converged scenes stay cheap.  The scene's first block may set this flag
  // during this launch (below), so the wave takes one value for all its lanes; a wave that
  // still sees 0 finds the same convergence test true and returns before any barrier.
  if (__builtin_amdgcn_readfirstlane(V.pdone[s])) return;
  const T* Prz_cur = parity ? B.P_rz1 : B.P_rz0;
  const T* Prz_old = parity ? B.P_rz0 : B.P_rz1;
  const T* pold = parity ? B.p1 : B.p0;
  T* pnew = parity ? B.p0 : B.p1;
  const T* sval = reinterpret_cast<const T*>(V.val);
  const int sub = threadIdx.x & (kRowLanes - 1);
  const int row = TS.b0[blk] + (int)(threadIdx.x / kRowLanes);
  const bool inrange = row < TS.b1[blk];
  // row data first, none of it behind another load (the free flag only masks the ranges)
  int fr = 0, rp0 = 0, rp1 = 0, dp0 = 0, dp1 = 0;
  if (inrange) {
    fr = V.nfree[row];
    rp0 = V.rowptr[row];
    rp1 = V.rowptr[row + 1];
    dp0 = B.drowptr[row];
    dp1 = B.drowptr[row + 1];
  }
  const bool live = inrange && fr;
  const int k0 = live ? rp0 : 0, k1 = live ? rp1 : 0;
  const int d0 = live ? dp0 : 0, d1 = live ? dp1 : 0;
  // the row's last lane owns its results; its own entries of z and p_{k-1}, and the rest
  // offset and weight for the restriction of q, depend on nothing but the row: loaded first
  const bool owner = inrange && sub == kRowLanes - 1;
  T dr[4] = {(T)0, (T)0, (T)0, (T)0};
  T zr[3] = {(T)0, (T)0, (T)0}, por[3] = {(T)0, (T)0, (T)0};
  if (owner) {
    if (B.cg_on)
      for (int c = 0; c < 4; ++c) dr[c] = B.cg_dw[4 * row + c];
    for (int c = 0; c < 3; ++c) {
      zr[c] = B.z[3 * row + c];
      por[c] = pold[3 * row + c];
    }
  }
  // the lane's first static block with its operands
  const bool has_s = k0 + sub < k1;
  SpmvEntry<T> es;
  if (has_s) spmv_load(sval, V.col, B.z, pold, k0 + sub, es);
  T rzc, rzo, gg;
  {
    const int lane = threadIdx.x & (kWave - 1);
    const int b0 = TN.sblk[s], b1 = TN.sblk[s + 1];
    const T* const P[3] = {Prz_cur, Prz_old, B.P_gg};
    T v[3];
    strided_sums<2>(P, {b0, b0, b0}, {b1, b1, b1}, lane, v);
    wave_total_n(v);
    rzc = v[0];
    rzo = v[1];
    gg = v[2];
  }
  // the relative tolerance: fixed, or the forcing term of this Newton iteration (every wave
  // computes the same value from the same sums)
  const T eta = (T)(V.sc[s].forcing ? forcing_eta(V.sc[s].pcg_eta, (double)gg, B.ggprev[s], B.etaprev[s])
                                    : V.sc[s].pcg_eta);
  // iters[s] is only written by k_pcg_update, so every wave sees the same count here
  // Stop once r^T M^{-1} r <= eta^2 g^T D^{-1} g: the residual measured in the
  // preconditioner's norm, so that a few stiff unknowns (a body held by its constraint
  // penalty) do not set the scale for all the others.
  const bool conv = (rzc <= eta * eta * gg) || !(rzc > (T)0) || !(rzo > (T)0) || B.iters[s] >= B.max_iters ||
                    B.indef[s];
  if (conv) {
    if (blk == TS.sblk[s] && threadIdx.x == 0) V.pdone[s] = 1;
    return;
  }
  const T beta = rzc / rzo;
  T q0 = (T)0, q1 = (T)0, q2 = (T)0;
  // blocks in the order of a plain strided pass: static range, then dynamic range
  if (has_s) spmv_acc(es, beta, q0, q1, q2);
  for (int k = k0 + sub + kRowLanes; k < k1; k += kRowLanes) {
    spmv_load(sval, V.col, B.z, pold, k, es);
    spmv_acc(es, beta, q0, q1, q2);
  }
  for (int k = d0 + sub; k < d1; k += kRowLanes) {
    spmv_load(B.dval, B.dcol, B.z, pold, k, es);
    spmv_acc(es, beta, q0, q1, q2);
  }
  q0 = row16_total(q0);
  q1 = row16_total(q1);
  q2 = row16_total(q2);
  T pq = (T)0;
  if (owner) {
    T pn[3];
    for (int c = 0; c < 3; ++c) {
      pn[c] = zr[c] + beta * por[c];
      pnew[3 * row + c] = pn[c];
    }
    B.q[3 * row] = q0;
    B.q[3 * row + 1] = q1;
    B.q[3 * row + 2] = q2;
    if (live) pq = pn[0] * q0 + pn[1] * q1 + pn[2] * q2;
  }
  if (!B.cg_on) {
    __shared__ T red[TPB / kWave];
    {
      T one[1] = {pq};
      block_total256_n(one, red);
      pq = one[0];
    }
    if (threadIdx.x == 0) B.P_pq[blk] = pq;
    return;
  }
  // restriction of q onto the rigid modes of the rows' aggregate: (sum q, sum d x q)
  T v[7] = {pq, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0};
  if (owner) {
    v[1] = dr[3] * q0;
    v[2] = dr[3] * q1;
    v[3] = dr[3] * q2;
    v[4] = dr[1] * q2 - dr[2] * q1;
    v[5] = dr[2] * q0 - dr[0] * q2;
    v[6] = dr[0] * q1 - dr[1] * q0;
  }
  __shared__ T red7[7 * (TPB / kWave)];
  block_total256_n(v, red7);
  if (threadIdx.x == 0) {
    B.P_pq[blk] = v[0];
    for (int k = 0; k < 6; ++k) B.P_qc[6 * blk + k] = v[1 + k];
  }
}

// NT threads per 64-node block: 256 in general (the coarse entries of a scene spread over 4
// wavefronts), 64 when no scene has more than 64 coarse entries (one wavefront per block does
// all the work; with at most 64 entries the 256-thread form holds them all in its first
// wavefront and adds exact zeros from the others, so both forms give the same bits).
template <class T, int NT>
__global__ void __launch_bounds__(NT) k_pcg_update(View V, BlockTable TN, BlockTable TS,
                                                   PcgBufsT<T> B, int parity) {
  static_assert(NT == kWave || NT == TPB, "one or four wavefronts per block");
  const int blk = xcd_block(TN.nblk);
  if (blk < 0) return;
  __shared__ T rs[kWave][3];
  __shared__ T red[NT / kWave][6];
  const int s = TN.sc[blk];
  if (V.pdone[s]) return;  // one uniform load: the blocks of converged scenes stay cheap
  const int wid = (int)threadIdx.x / kWave, lane = (int)threadIdx.x % kWave;
  const T* Prz_cur = parity ? B.P_rz1 : B.P_rz0;
  T* Prz_new = parity ? B.P_rz0 : B.P_rz1;
  const T* pk = parity ? B.p0 : B.p1;
  // Every load that does not depend on alpha is issued first, so their latencies overlap
  // instead of adding up.
  // ---- node operands (wave 0: one node per lane)
  const int n0 = TN.b0[blk], n1 = TN.b1[blk];
  const int n = n0 + lane;
  const bool live = wid == 0 && n < n1;
  T pkn[3] = {(T)0, (T)0, (T)0}, qn[3] = {(T)0, (T)0, (T)0}, rn[3] = {(T)0, (T)0, (T)0};
  T P9[9] = {(T)0, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0, (T)0};
  double dxn[3] = {0.0, 0.0, 0.0};
  int ntn = 0, nfn = 0;
  if (live) {
    ntn = V.ntype[n];
    nfn = V.nfree[n];
    for (int c = 0; c < 3; ++c) {
      pkn[c] = pk[3 * n + c];
      qn[c] = B.q[3 * n + c];
      rn[c] = B.r[3 * n + c];
      dxn[c] = B.dx[3 * n + c];
    }
    for (int i = 0; i < 9; ++i) P9[i] = B.pinv[9 * (size_t)n + i];
  }
  // ---- coarse operands (4 waves share the scene's coarse entries)
  constexpr int kPerThread = NT == kWave ? 1 : 6 * kCoarseMaxAgg / TPB;
  const int a = B.cg_on ? B.cg_blk_agg[blk] : -1;
  int m = 0, la = 0;
  T rcj[kPerThread], qsj[kPerThread];
  float Aij[kPerThread][6];
  T dn[3] = {(T)0, (T)0, (T)0};
  T* rc_next = nullptr;
  if (a >= 0) {
    const int a0 = B.cg_sc_a0[s];
    m = B.cg_sc_m[s];
    la = a - a0;
    const T* rc_cur = (parity ? B.cg_rca1 : B.cg_rca0) + 6 * (size_t)a0;
    rc_next = (parity ? B.cg_rca0 : B.cg_rca1) + 6 * (size_t)a0;
    const float* Ai = B.cg_ainv + B.cg_sc_off[s] + (size_t)6 * la * m;
    // TS blocks of aggregate j / 6: runs of tsn blocks from the scene's first one
    const int ts0 = B.cg_sc_ts0[s], tsn = B.cg_sc_tsn[s], tsend = B.cg_sc_tsend[s];
    // Loads without branches: entries past m read entry 0 (in range) and are weighted 0, and
    // the 4 partials of an aggregate of one block are read at once, so nothing waits until
    // every operand of the thread is in flight.
    T qv[kPerThread][4];
    bool on[kPerThread];
#pragma unroll
    for (int t = 0; t < kPerThread; ++t) {
      const int j = (int)threadIdx.x + NT * t;
      on[t] = j < m;
      const int jj = on[t] ? j : 0;
      const int k = jj % 6, i0 = ts0 + tsn * (jj / 6), i1 = min(i0 + tsn, tsend);
      rcj[t] = rc_cur[jj];
#pragma unroll
      for (int u = 0; u < 4; ++u) qv[t][u] = B.P_qc[6 * min(i0 + u, i1 - 1) + k];
#pragma unroll
      for (int q = 0; q < 6; ++q) Aij[t][q] = Ai[(size_t)q * m + jj];
      // aggregates of more than one block: the remaining partials, four at a time
      T extra = (T)0;
      for (int ib = i0 + 4; ib < i1; ib += 4) {
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = ib + u < i1 ? B.P_qc[6 * (ib + u) + k] : (T)0;
        extra += v[0];
        extra += v[1];
        extra += v[2];
        extra += v[3];
      }
      qsj[t] = extra;
      for (int u = 0; u < 4; ++u)
        if (i0 + u >= i1) qv[t][u] = (T)0;
    }
#pragma unroll
    for (int t = 0; t < kPerThread; ++t) {
      // same order as one pass over the aggregate's partials
      T qs = (T)0;
      qs += qv[t][0];
      qs += qv[t][1];
      qs += qv[t][2];
      qs += qv[t][3];
      qsj[t] = qs + qsj[t];
      if (!on[t]) {
        rcj[t] = qsj[t] = (T)0;
        for (int q = 0; q < 6; ++q) Aij[t][q] = 0.f;
      }
    }
    if (live)
      for (int c = 0; c < 3; ++c) dn[c] = B.cg_d[3 * n + c];
  }
  // ---- scene scalars (every wave computes them itself)
  const T* const Ptot[2] = {Prz_cur, B.P_pq};
  T tot[2];
  strided_sums<4>(Ptot, {TN.sblk[s], TS.sblk[s]}, {TN.sblk[s + 1], TS.sblk[s + 1]}, lane, tot);
  wave_total_n(tot);
  const T rzs = tot[0], pqs = tot[1];
  const T alpha = pqs > (T)0 ? rzs / pqs : (T)0;
  // a direction of non-positive curvature: the system is not positive definite (CG stops;
  // the next sparse product sees the flag, written only here, in the scene's first block)
  if (!(pqs > (T)0) && rzs > (T)0 && blk == TN.sblk[s] && threadIdx.x == 0) B.indef[s] = 1;
  // ---- node update: x += alpha p, r -= alpha q, z = D^{-1} r
  T r[3] = {(T)0, (T)0, (T)0};
  if (live) {
    for (int c = 0; c < 3; ++c) r[c] = rn[c] - alpha * qn[c];
    for (int c = 0; c < 3; ++c) {
      B.dx[3 * n + c] = dxn[c] + (double)(alpha * pkn[c]);
      B.r[3 * n + c] = r[c];
    }
  }
  if (wid == 0)
    for (int c = 0; c < 3; ++c) rs[lane][c] = r[c];
  __syncthreads();
  T z[3] = {(T)0, (T)0, (T)0};
  if (live && nfn) {
    if (ntn == 0) {
      for (int i = 0; i < 3; ++i) z[i] = P9[3 * i] * r[0] + P9[3 * i + 1] * r[1] + P9[3 * i + 2] * r[2];
    } else {
      precond_apply<T>(V, B.pinv, n, n0, rs, z);
    }
  }
  if (a >= 0) {
    // r_c,k+1 = r_c,k - alpha P^T q_k; e = rows of A_c^{-1} for the block's aggregate times it
    const bool first = blk == B.cg_agg_b0[a];  // writes the aggregate's entries of r_c,k+1
    T e[6] = {(T)0, (T)0, (T)0, (T)0, (T)0, (T)0};
#pragma unroll
    for (int t = 0; t < kPerThread; ++t) {
      const T rj = rcj[t] - alpha * qsj[t];
      const int j = (int)threadIdx.x + NT * t;
      if (first && j < m && j / 6 == la) rc_next[j] = rj;
#pragma unroll
      for (int q = 0; q < 6; ++q) e[q] += (T)Aij[t][q] * rj;
    }
    wave_total_n(e);
    if constexpr (NT == TPB) {
      if (lane == 0)
        for (int q = 0; q < 6; ++q) red[wid][q] = e[q];
      __syncthreads();
      for (int q = 0; q < 6; ++q) e[q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
    }
    if (live && ntn == 0 && nfn) {
      z[0] += e[0] + (e[4] * dn[2] - e[5] * dn[1]);
      z[1] += e[1] + (e[5] * dn[0] - e[3] * dn[2]);
      z[2] += e[2] + (e[3] * dn[1] - e[4] * dn[0]);
    }
  }
  if (wid != 0) return;
  if (live)
    for (int c = 0; c < 3; ++c) B.z[3 * n + c] = z[c];
  // block partial of r.z (z with its coarse part)
  const T rz = wave_total(r[0] * z[0] + r[1] * z[1] + r[2] * z[2]);
  if (lane == 0) {
    Prz_new[blk] = rz;
    if (blk == TN.sblk[s]) ++B.iters[s];
  }
}

// Coarse correction of z_0, one wave per 64-node block: the scene's restricted residual r_c
// (sum of block partials per aggregate), e = rows of A_c^{-1} for the block's aggregate
// times r_c, z += t + w x d on the block's soft nodes, and r_c . e of the aggregate added to
// the partial of r.z of the aggregate's first block.
template <class T>
__global__ void __launch_bounds__(kWave) k_pcg_coarse(View V, BlockTable TN, PcgBufsT<T> B, T* prz) {
  constexpr int kPerLane = 6 * kCoarseMaxAgg / kWave;  // coarse entries per lane (at most)
  const int blk = xcd_block(TN.nblk);
  if (blk < 0) return;
  const int s = TN.sc[blk];
  if (V.pdone[s]) return;
  const int a = B.cg_blk_agg[blk];
  if (a < 0) return;
  const int a0 = B.cg_sc_a0[s], m = B.cg_sc_m[s], la = a - a0;
  const int lane = threadIdx.x;
  // the block's own node (issued early: independent of the coarse solve)
  const int n = TN.b0[blk] + lane;
  const bool mine = n < TN.b1[blk] && V.ntype[n] == 0 && V.nfree[n];
  T dn[3] = {(T)0, (T)0, (T)0};
  if (mine)
    for (int c = 0; c < 3; ++c) dn[c] = B.cg_d[3 * n + c];
  // e = rows 6 la .. 6 la + 5 of A_c^{-1} times r_c; lane j-slices of r_c summed from the
  // block partials of their aggregates
  const float* Ai = B.cg_ainv + B.cg_sc_off[s] + (size_t)6 * la * m;
  // aggregates are runs of grp consecutive blocks from the scene's first block sb (the last
  // run may be shorter), so a lane's block indices are plain arithmetic
  const int sb = B.cg_agg_b0[a0], grp = B.cg_agg_b1[a0] - sb, send = B.cg_agg_b1[a0 + m / 6 - 1];
  T e[6] = {(T)0, (T)0, (T)0, (T)0, (T)0, (T)0};
#pragma unroll
  for (int t = 0; t < kPerLane; ++t) {
    const int j = lane + kWave * t;
    if (j < m) {
      const int b0 = sb + (j / 6) * grp, b1 = min(b0 + grp, send), k = j % 6;
      T rj = B.cg_rc[6 * b0 + k];
      for (int b = b0 + 1; b < b1; ++b) rj += B.cg_rc[6 * b + k];
#pragma unroll
      for (int r = 0; r < 6; ++r) e[r] += (T)Ai[(size_t)r * m + j] * rj;
    }
  }
  wave_total_n(e);
  if (lane == 0 && blk == B.cg_agg_b0[a]) {
    T dot = (T)0;
    for (int k = 0; k < 6; ++k) {
      T rk = (T)0;
      for (int b = B.cg_agg_b0[a]; b < B.cg_agg_b1[a]; ++b) rk += B.cg_rc[6 * b + k];
      dot += rk * e[k];
      B.cg_rca0[6 * (size_t)a + k] = rk;  // r_c,0 for the recurrence of the iterations
    }
    prz[blk] += dot;
  }
  if (mine) {
    B.z[3 * n] += e[0] + (e[4] * dn[2] - e[5] * dn[1]);
    B.z[3 * n + 1] += e[1] + (e[5] * dn[0] - e[3] * dn[2]);
    B.z[3 * n + 2] += e[2] + (e[3] * dn[1] - e[4] * dn[0]);
  }
}

// ------------------------------------------------------------------ FP32 PCG, FP64 refinement
__global__ void k_to_f32(size_t n, const double* src, float* dst) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

// gres = g + H dx on the free rows (16 lanes per block-row, as the sparse product of the
// PCG), zero on the others; scenes with pdone set are left alone.  With H dx = -g solved
// exactly gres would vanish: it is the FP64 residual of the FP32 passes' solution.
__global__ void __launch_bounds__(TPB) k_refine_resid(View V, BlockTable TS, const int* drowptr,
                                                      const int* dcol, const double* dval,
                                                      const double* g, const double* dx, double* gres) {
  const int blk = xcd_block(TS.nblk);
  if (blk < 0) return;
  const int s = TS.sc[blk];
  if (V.pdone[s]) return;  // set by the host before the launch: uniform over the workgroup
  const int sub = threadIdx.x & (kRowLanes - 1);
  const int row = TS.b0[blk] + (int)(threadIdx.x / kRowLanes);
  const bool inrange = row < TS.b1[blk];
  const bool live = inrange && V.nfree[row];
  double q0 = 0.0, q1 = 0.0, q2 = 0.0;
  if (live) {
    for (int k = V.rowptr[row] + sub; k < V.rowptr[row + 1]; k += kRowLanes) {
      const double* A = V.val + 9 * (size_t)k;
      const double* x = dx + 3 * (size_t)V.col[k];
      q0 += A[0] * x[0] + A[1] * x[1] + A[2] * x[2];
      q1 += A[3] * x[0] + A[4] * x[1] + A[5] * x[2];
      q2 += A[6] * x[0] + A[7] * x[1] + A[8] * x[2];
    }
    for (int k = drowptr[row] + sub; k < drowptr[row + 1]; k += kRowLanes) {
      const double* A = dval + 9 * (size_t)k;
      const double* x = dx + 3 * (size_t)dcol[k];
      q0 += A[0] * x[0] + A[1] * x[1] + A[2] * x[2];
      q1 += A[3] * x[0] + A[4] * x[1] + A[5] * x[2];
      q2 += A[6] * x[0] + A[7] * x[1] + A[8] * x[2];
    }
  }
  q0 = row16_total(q0);
  q1 = row16_total(q1);
  q2 = row16_total(q2);
  if (inrange && sub == kRowLanes - 1) {
    gres[3 * (size_t)row] = live ? g[3 * (size_t)row] + q0 : 0.0;
    gres[3 * (size_t)row + 1] = live ? g[3 * (size_t)row + 1] + q1 : 0.0;
    gres[3 * (size_t)row + 2] = live ? g[3 * (size_t)row + 2] + q2 : 0.0;
  }
}

// Per TN block (one wavefront): gres^T D^-1 gres and g^T D^-1 g over its free nodes, with the
// FP64 block-Jacobi inverse D^-1 (3x3 per soft node, 12x12 per affine body).
__global__ void __launch_bounds__(kWave) k_refine_norm(View V, BlockTable TN, const double* pinv,
                                                       const double* g, const double* gres, double* part) {
  const int blk = xcd_block(TN.nblk);
  if (blk < 0) return;
  __shared__ double rs[kWave][3], gs[kWave][3];
  const int s = TN.sc[blk];
  if (V.pdone[s]) return;  // set by the host before the launch: uniform over the wavefront
  const int n0 = TN.b0[blk];
  const int n = n0 + (int)threadIdx.x;
  const bool live = n < TN.b1[blk];
  const bool f = live && V.nfree[n];
  for (int c = 0; c < 3; ++c) {
    rs[threadIdx.x][c] = f ? gres[3 * (size_t)n + c] : 0.0;
    gs[threadIdx.x][c] = f ? g[3 * (size_t)n + c] : 0.0;
  }
  __syncthreads();
  double zr[3] = {0.0, 0.0, 0.0}, zg[3] = {0.0, 0.0, 0.0};
  if (live) {
    precond_apply<double>(V, pinv, n, n0, rs, zr);
    precond_apply<double>(V, pinv, n, n0, gs, zg);
  }
  const int l = threadIdx.x;
  double v[2] = {rs[l][0] * zr[0] + rs[l][1] * zr[1] + rs[l][2] * zr[2],
                 gs[l][0] * zg[0] + gs[l][1] * zg[1] + gs[l][2] * zg[2]};
  wave_total_n(v);
  if (threadIdx.x == 0) {
    part[2 * (size_t)blk] = v[0];
    part[2 * (size_t)blk + 1] = v[1];
  }
}

// dx = c (first pass) or dx += c on the nodes of the scenes solved in this call (act):
// the other scenes' directions are left as they are
__global__ void k_refine_apply(View V, const double* c, double* dx, int assign) {
  const int i = gid();
  if (i >= 3 * V.Nn || !V.act[V.nscene[i / 3]]) return;
  dx[i] = assign ? c[i] : dx[i] + c[i];
}

// Number of active pairs per scene (statistics).
__global__ void k_count_scene(int n, const int* pscene, int* cnt) {
  const int k = gid();
  if (k < n) atomicAdd(cnt + pscene[k], 1);
}

// ------------------------------------------------------------------ convergence & CCD
// Largest displacement component of the Newton direction per scene: free soft vertices and
// affine-body vertices (J p).  Lanes of a wave that share a scene combine before the atomic.
__global__ void k_pmax(View V, const double* p, unsigned long long* pmax) {
  const int k = gid();
  double m = 0.0;
  int s = -1;
  if (k < V.Nn) {
    const int n = k;
    if (V.ntype[n] == 0 && V.nfree[n] && V.act[V.nscene[n]]) {
      m = fmax(fabs(p[3 * n]), fmax(fabs(p[3 * n + 1]), fabs(p[3 * n + 2])));
      if (isnan(p[3 * n]) || isnan(p[3 * n + 1]) || isnan(p[3 * n + 2])) m = INFINITY;
      s = V.nscene[n];
    }
  } else if (k - V.Nn < V.Ncv) {
    const int cv = k - V.Nn;
    const int b = V.cvb[cv];
    if (b >= 0 && !V.bsnap[b] && V.act[V.bscene[b]]) {
      double d[3];
      body_point(V, p + 3 * V.bnode[b], cv, d);
      m = fmax(fabs(d[0]), fmax(fabs(d[1]), fabs(d[2])));
      if (isnan(d[0]) || isnan(d[1]) || isnan(d[2])) m = INFINITY;
      s = V.bscene[b];
    }
  }
  // wave-uniform scene: reduce in registers, one atomic per wave
  const int s0 = __shfl(s, 0, 64);
  const bool uniform = __all(s == s0);
  if (uniform) {
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0 && s0 >= 0) atomic_max_pos(pmax + s0, m);
  } else if (s >= 0) {
    atomic_max_pos(pmax + s, m);
  }
}

__global__ void k_ccd(View V, int n, const int* cq, const int* ct, unsigned long long* amin) {
  const int k = gid();
  if (k >= n) return;
  int ids[4];
  const int kind = cand_verts(V, cq[k], ct[k], ids);
  double x12[12], p12[12];
  gather12(V.cpos, ids, x12);
  gather12(V.cdisp, ids, p12);
  unsigned long long* am = amin + V.qscene[cq[k]];
  const double t = accd(kind, x12, p12, 0.1, 100000, am);
  // the minimum starts at 1 and most pairs return 1: only smaller bounds contend for it
  if (t < 1.0) atomic_min_pos(am, t);
}

// off[s] = first candidate of scene s (candidates are sorted by scene); off[S] = n.
__global__ void k_scene_offsets(View V, int n, const int* cq, int* off) {
  const int k = gid();
  if (k > n) return;
  const int cur = k < n ? V.qscene[cq[k]] : V.S;
  const int prev = k > 0 ? V.qscene[cq[k - 1]] : -1;
  for (int s = prev + 1; s <= cur; ++s) off[s] = k;
}

// ------------------------------------------------------------------ line search
__device__ __forceinline__ double trial_alpha(const double* abase, int s, int k) {
  return ldexp(abase[s], -k);
}

__global__ void __launch_bounds__(kWave) k_ls_nodes(View V, BlockTable T, LsBufs L) {
  const int s = T.sc[blockIdx.x];
  if (!V.act[s]) return;
  const int n = T.b0[blockIdx.x] + threadIdx.x;
  double pe = 0.0, pp = 0.0, m = 0.0;
  if (n < T.b1[blockIdx.x] && V.ntype[n] == 0 && V.nfree[n]) {
    m = V.mass[n];
    for (int c = 0; c < 3; ++c) {
      const double pc = L.p[3 * n + c];
      pe += pc * (V.x[3 * n + c] - V.xhat[3 * n + c]);
      pp += pc * pc;
    }
  }
  for (int k = 0; k < kTrials; ++k) {
    const double a = trial_alpha(L.abase, s, k);
    const double dE = wave_sum(0.5 * m * (2.0 * a * pe + a * a * pp));
    if (threadIdx.x == 0) L.part_nodes[kTrials * blockIdx.x + k] = dE;
  }
}

__global__ void __launch_bounds__(TPB) k_ls_tets(View V, BlockTable T, LsBufs L) {
  __shared__ double red[4];
  const int s = T.sc[blockIdx.x];
  if (!V.act[s]) return;
  const SceneConst& sc = V.sc[s];
  const int t = T.b0[blockIdx.x] + threadIdx.x;
  const bool live = t < T.b1[blockIdx.x];
  double x12[12], p12[12], Dm[9], e0 = 0.0, scale = 0.0;
  if (live) {
    for (int v = 0; v < 4; ++v) {
      const int node = V.tv[v * V.Nt + t];
      for (int c = 0; c < 3; ++c) {
        x12[3 * v + c] = V.x[3 * node + c];
        p12[3 * v + c] = L.p[3 * node + c];
      }
    }
    for (int k = 0; k < 9; ++k) Dm[k] = V.Dminv[k * V.Nt + t];
    double F[9];
    deformation_gradient(x12, Dm, F);
    e0 = nh_density(F, sc.mu, sc.lam);
    scale = sc.h * sc.h * V.tvol[t];
  }
  int bad = 0;
  for (int k = 0; k < kTrials; ++k) {
    double dE = 0.0;
    if (live) {
      const double a = trial_alpha(L.abase, s, k);
      double xt[12], F[9];
      for (int i = 0; i < 12; ++i) xt[i] = x12[i] + a * p12[i];
      deformation_gradient(xt, Dm, F);
      const double e = nh_density(F, sc.mu, sc.lam);
      if (isinf(e)) bad |= 1 << k;
      else dE = scale * (e - e0);
    }
    dE = block_sum256(dE, red);
    if (threadIdx.x == 0) L.part_tets[kTrials * blockIdx.x + k] = dE;
  }
  if (bad) atomicOr(L.infeasible + s, bad);
}

__device__ double body_energy(const View& V, int b, const double* y, const SceneConst& sc) {
  const double* bm = V.bmass + 10 * b;
  const double* yh = V.xhat + 3 * V.bnode[b];
  double dy[12], My[12];
  for (int k = 0; k < 12; ++k) dy[k] = y[k] - yh[k];
  my_apply(bm, dy, My);
  double e = 0.0;
  for (int k = 0; k < 12; ++k) e += 0.5 * dy[k] * My[k];
  double A[9], gA[9], ea;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[3 * i + j] = y[3 + 3 * j + i];
  Modes m;
  arap_modes(A, m, &ea, gA);
  e += sc.h * sc.h * sc.kappa_s * V.bvol[b] * ea;
  if (V.bpres[b]) {
    double c[12], Mc[12];
    for (int k = 0; k < 12; ++k) c[k] = y[k] - V.bstar[12 * b + k];
    my_apply(bm, c, Mc);
    double cc = 0.0, lc = 0.0;
    for (int k = 0; k < 12; ++k) {
      cc += c[k] * Mc[k];
      lc += V.blam[12 * b + k] * Mc[k];
    }
    e += 0.5 * V.bkap[b] * cc - lc;
  }
  return e;
}

// Bodies and contact pairs: one thread per (element, trial) with trial index 0 for the
// current point and 1 + k for step size k; the energy differences are formed by the
// reduction (the current point's energy is finite by construction).
constexpr int kLsSlots = kTrials + 1;
__global__ void k_ls_bodies(View V, LsBufs L) {
  const int g = gid();
  const int b = g / kLsSlots, slot = g % kLsSlots;
  if (b >= V.Nb) return;
  const int s = V.bscene[b];
  if (!V.act[s] || V.bsnap[b]) {
    L.e_bodies[kLsSlots * b + slot] = 0.0;
    return;
  }
  const SceneConst& sc = V.sc[s];
  const double* y = V.x + 3 * V.bnode[b];
  const double* p = L.p + 3 * V.bnode[b];
  const double a = slot == 0 ? 0.0 : trial_alpha(L.abase, s, slot - 1);
  double yt[12];
  for (int i = 0; i < 12; ++i) yt[i] = slot == 0 ? y[i] : y[i] + a * p[i];
  L.e_bodies[kLsSlots * b + slot] = body_energy(V, b, yt, sc);
}

__global__ void k_ls_pairs(View V, int n, const int* cq, const int* ct, LsBufs L) {
  const int g = gid();
  const int k = g / kLsSlots, slot = g % kLsSlots;
  if (k >= n) return;
  const int s = V.qscene[cq[k]];
  const SceneConst& sc = V.sc[s];
  int ids[4];
  const int kind = cand_verts(V, cq[k], ct[k], ids);
  double x12[12], p12[12];
  gather12(V.cpos, ids, x12);
  gather12(V.cdisp, ids, p12);
  const double meps = kind == 1 ? 1e-3 * V.elen2[V.qidx[cq[k]]] * V.elen2[ct[k]] : 0.0;
  const double kap = sc.h * sc.h * sc.kappa;
  double e;
  if (slot == 0) {
    e = barrier_energy(kind, x12, meps, sc.dhat, kap);
  } else {
    const double a = trial_alpha(L.abase, s, slot - 1);
    double xt[12];
    for (int i = 0; i < 12; ++i) xt[i] = x12[i] + a * p12[i];
    e = barrier_energy(kind, xt, meps, sc.dhat, kap);
    if (isinf(e)) atomicOr(L.infeasible + s, 1 << (slot - 1));
  }
  L.e_pairs[kLsSlots * (size_t)k + slot] = e;
}

// Friction energies mu lambda h^2 f0(|u|) at the current point and the 8 trials.
__global__ void k_ls_fric(View V, LsBufs L) {
  const int g = gid();
  const int k = g / kLsSlots, slot = g % kLsSlots;
  if (k >= L.F.n) return;
  int ids[4];
  double w[4];
  for (int v = 0; v < 4; ++v) {
    ids[v] = L.F.v[4 * k + v];
    w[v] = L.F.w[4 * k + v];
  }
  const int s = V.cvscene[ids[0]];
  const SceneConst& sc = V.sc[s];
  double x12[12], p12[12];
  gather12(V.cpos, ids, x12);
  gather12(V.cdisp, ids, p12);
  if (slot > 0) {
    const double a = trial_alpha(L.abase, s, slot - 1);
    for (int i = 0; i < 12; ++i) x12[i] += a * p12[i];
  }
  const d3 u = friction_u(x12, w, ld(L.F.c0 + 3 * k), ld(L.F.nrm + 3 * k));
  L.e_fric[kLsSlots * (size_t)k + slot] = sc.h * sc.h * L.F.mul[k] * friction_f0(sqrt(dot(u, u)), sc.eh);
}

// Energy differences of the swept pairs summed per block of one scene's candidates.
__global__ void __launch_bounds__(TPB) k_ls_pair_sums(View V, BlockTable TP, LsBufs L) {
  __shared__ double red[TPB / kWave][kTrials];
  const int s = TP.sc[blockIdx.x];
  if (!V.act[s]) return;
  const int t = threadIdx.x;
  double acc[kTrials];
  for (int k = 0; k < kTrials; ++k) acc[k] = 0.0;
  for (int c = TP.b0[blockIdx.x] + t; c < TP.b1[blockIdx.x]; c += TPB) {
    const double* e = L.e_pairs + kLsSlots * (size_t)c;
    for (int k = 0; k < kTrials; ++k) acc[k] += isinf(e[1 + k]) ? 0.0 : e[1 + k] - e[0];
  }
  wave_sum_n(acc);
  if ((t & (kWave - 1)) == 0)
    for (int k = 0; k < kTrials; ++k) red[t / kWave][k] = acc[k];
  __syncthreads();
  if (t < kTrials)
    L.part_pairs[kTrials * blockIdx.x + t] = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
}

// Per scene: dE[k] = sum over the scene's node, tet and pair-block partials and its bodies,
// all 8 trials in one pass (fixed assignment and order, so the sums are deterministic).
__global__ void __launch_bounds__(TPB) k_ls_reduce(View V, BlockTable TN, BlockTable TT, BlockTable TP,
                                                   LsBufs L) {
  __shared__ double red[TPB / kWave][kTrials];
  const int s = blockIdx.x;
  if (!V.act[s]) return;
  const int t = threadIdx.x;
  double acc[kTrials];
  for (int k = 0; k < kTrials; ++k) acc[k] = 0.0;
  for (int b = TN.sblk[s] + t; b < TN.sblk[s + 1]; b += TPB)
    for (int k = 0; k < kTrials; ++k) acc[k] += L.part_nodes[kTrials * b + k];
  for (int b = TT.sblk[s] + t; b < TT.sblk[s + 1]; b += TPB)
    for (int k = 0; k < kTrials; ++k) acc[k] += L.part_tets[kTrials * b + k];
  for (int b = V.sc[s].body0 + t; b < V.sc[s].body1; b += TPB) {
    const double* e = L.e_bodies + kLsSlots * b;
    for (int k = 0; k < kTrials; ++k) acc[k] += e[1 + k] - e[0];
  }
  for (int b = TP.sblk[s] + t; b < TP.sblk[s + 1]; b += TPB)
    for (int k = 0; k < kTrials; ++k) acc[k] += L.part_pairs[kTrials * b + k];
  if (L.F.n > 0)
    for (int b = L.F.soff[s] + t; b < L.F.soff[s + 1]; b += TPB) {
      const double* e = L.e_fric + kLsSlots * (size_t)b;
      for (int k = 0; k < kTrials; ++k) acc[k] += e[1 + k] - e[0];
    }
  wave_sum_n(acc);
  if ((t & (kWave - 1)) == 0)
    for (int k = 0; k < kTrials; ++k) red[t / kWave][k] = acc[k];
  __syncthreads();
  if (t < kTrials) L.dE[kTrials * s + t] = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
}

__global__ void k_update(View V, const double* p, const double* alpha) {
  const int n = gid();
  if (n >= V.Nn) return;
  const int s = V.nscene[n];
  if (!V.act[s] || !V.nfree[n]) return;
  const double a = alpha[s];
  for (int c = 0; c < 3; ++c) V.x[3 * n + c] += a * p[3 * n + c];
}

// action: 0 none, 1 snap onto the target, 2 multiplier update, 3 update and double kappa
__global__ void k_al_apply(View V, const int* action) {
  const int b = gid();
  if (b >= V.Nb) return;
  const int act = action[b];
  if (act == 0) return;
  const int n0 = V.bnode[b];
  if (act == 1) {
    for (int k = 0; k < 12; ++k) V.x[3 * n0 + k] = V.bstar[12 * b + k];
    V.bsnap[b] = 1;
    for (int u = 0; u < 4; ++u) V.nfree[n0 + u] = 0;
    return;
  }
  const double kap = V.bkap[b];
  for (int k = 0; k < 12; ++k) V.blam[12 * b + k] -= kap * (V.x[3 * n0 + k] - V.bstar[12 * b + k]);
  if (act == 3) V.bkap[b] = 2.0 * kap;
}

// Start of a step: penalty reset, every body unsnapped (its 4 pseudo-nodes become unknowns
// again).  The multipliers carry over from the previous accepted step (they approximate the
// constraint force, which changes little from one step to the next); they start at zero, and
// a failed step or a state write clears them (k_body_clear_lambda).
__global__ void k_body_reset(View V, double kappa0) {
  const int b = gid();
  if (b >= V.Nb) return;
  V.bkap[b] = kappa0;
  V.bsnap[b] = 0;
  for (int u = 0; u < 4; ++u) V.nfree[V.bnode[b] + u] = 1;
}

// Multipliers of the bodies of the flagged scenes back to zero.
__global__ void k_body_clear_lambda(View V, const int* flag) {
  const int b = gid();
  if (b >= V.Nb || !flag[V.bscene[b]]) return;
  for (int k = 0; k < 12; ++k) V.blam[12 * b + k] = 0.0;
}

__global__ void k_velocity(View V, const int* ok) {
  const int n = gid();
  if (n >= V.Nn) return;
  const int s = V.nscene[n];
  if (!ok[s]) return;
  const double inv = 1.0 / V.sc[s].h;
  for (int c = 0; c < 3; ++c) V.v[3 * n + c] = (V.x[3 * n + c] - V.xn[3 * n + c]) * inv;
}

__global__ void k_rollback(View V, const int* failed) {
  const int n = gid();
  if (n >= V.Nn) return;
  if (!failed[V.nscene[n]]) return;
  for (int c = 0; c < 3; ++c) V.x[3 * n + c] = V.xn[3 * n + c];
}

// ------------------------------------------------------------------ debug evaluators
__global__ void k_debug_fem(int n, const double* x, const double* Dminv, const double* vol,
                            double mu, double lam, double* e, double* g, double* H, double* Hp) {
  const int t = gid();
  if (t >= n) return;
  const double* x12 = x + 12 * t;
  const double* Dm = Dminv + 9 * t;
  double F[9];
  deformation_gradient(x12, Dm, F);
  const double psi = nh_density(F, mu, lam);
  if (e) e[t] = vol[t] * psi;
  if (isinf(psi)) return;
  double P[9], w[12];
  nh_stress(F, mu, lam, P);
  pullback(P, Dm, vol[t], w);
  if (g)
    for (int i = 0; i < 12; ++i) g[12 * t + i] = w[i];
  Modes m;
  nh_modes(F, mu, lam, m);
  for (int pass = 0; pass < 2; ++pass) {
    double* out = pass == 0 ? H : Hp;
    if (!out) continue;
    out += 144 * (size_t)t;
    for (int i = 0; i < 144; ++i) out[i] = 0.0;
    for (int k = 0; k < 9; ++k) {
      const double lk = pass == 0 ? m.lam[k] : fmax(m.lam[k], 0.0);
      double Q[9];
      mode_matrix(m, k, Q);
      pullback(Q, Dm, 1.0, w);
      for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) out[12 * i + j] += vol[t] * lk * w[i] * w[j];
    }
  }
}

__global__ void __launch_bounds__(64) k_debug_barrier(int n, const int* kinds, const double* x,
                                                      const double* meps, double dhat, double kappa,
                                                      double* e, double* g, double* H, double* Hp,
                                                      int* types) {
  __shared__ WaveBarrierLds L;
  const int k = blockIdx.x;
  if (k >= n) return;
  double ee;
  int type;
  wave_barrier_derivs(kinds[k], x + 12 * k, meps[k], dhat, kappa, L, &ee, &type);
  if (threadIdx.x == 0) {
    if (e) e[k] = ee;
    if (types) types[k] = type;
  }
  if (g && threadIdx.x < 12) g[12 * k + threadIdx.x] = L.g[threadIdx.x];
  if (H)
    for (int i = threadIdx.x; i < 144; i += 64) H[144 * (size_t)k + i] = L.H[i];
  __syncthreads();
  wave_barrier_project(L);
  if (Hp)
    for (int i = threadIdx.x; i < 144; i += 64) Hp[144 * (size_t)k + i] = L.H[i];
}

__global__ void k_debug_ccd(int n, const int* kinds, const double* x, const double* p, double gap,
                            int max_iter, double* t) {
  const int k = gid();
  if (k >= n) return;
  t[k] = accd(kinds[k], x + 12 * k, p + 12 * k, gap, max_iter);
}

__global__ void k_debug_friction(int n, const int* kinds, const double* xn, const double* x,
                                 const double* meps, double dhat, double kappa, double mu,
                                 double eh, double* lam, double* e, double* g, double* H) {
  const int k = gid();
  if (k >= n) return;
  const double* xk = xn + 12 * (size_t)k;
  int type;
  const double s = pair_sqdist(kinds[k], xk, &type);
  double w[4];
  closest_point_weights(kinds[k], type, xk, w);
  d3 c = mk(0, 0, 0);
  for (int v = 0; v < 4; ++v) c = c + w[v] * ld(xk + 3 * v);
  const double cn = sqrt(dot(c, c));
  double* G = g + 12 * (size_t)k;
  double* Hk = H + 144 * (size_t)k;
  if (!(s > 0.0 && s < dhat * dhat && cn > 0.0)) {
    lam[k] = 0.0;
    e[k] = 0.0;
    for (int i = 0; i < 12; ++i) G[i] = 0.0;
    for (int i = 0; i < 144; ++i) Hk[i] = 0.0;
    return;
  }
  lam[k] = normal_force(kinds[k], xk, s, meps[k], dhat, kappa);
  e[k] = friction_derivs(x + 12 * (size_t)k, w, c, (1.0 / cn) * c, mu * lam[k], eh, G, Hk);
}

__global__ void k_debug_arap(int n, const double* A, double* e, double* g, double* H, double* Hp) {
  const int k = gid();
  if (k >= n) return;
  Modes m;
  double ee, gA[9];
  arap_modes(A + 9 * k, m, &ee, gA);
  if (e) e[k] = ee;
  if (g)
    for (int i = 0; i < 9; ++i) g[9 * k + i] = gA[i];
  for (int pass = 0; pass < 2; ++pass) {
    double* out = pass == 0 ? H : Hp;
    if (!out) continue;
    out += 81 * (size_t)k;
    for (int i = 0; i < 81; ++i) out[i] = 0.0;
    for (int q = 0; q < 9; ++q) {
      const double lk = pass == 0 ? m.lam[q] : fmax(m.lam[q], 0.0);
      double Q[9];
      mode_matrix(m, q, Q);
      for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j) out[9 * i + j] += lk * Q[i] * Q[j];
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers
#define LAUNCH(kern, n, tpb, s, ...)                                          \
  do {                                                                        \
    const int _nb = nblk((n), (tpb));                                         \
    if (_nb > 0) hipLaunchKernelGGL(kern, dim3(_nb), dim3(tpb), 0, s, __VA_ARGS__); \
  } while (0)

void launch_predict(const View& V, hipStream_t s) { LAUNCH(k_predict, V.Nn, TPB, s, V); }
void launch_set_moving(double* x, int n, const int* nodes, const double* tgt, hipStream_t s) {
  LAUNCH(k_set_moving, n, TPB, s, x, n, nodes, tgt);
}
void launch_touching(const View& V, int n, const int* cq, const int* ct, int* bad, hipStream_t s) {
  LAUNCH(k_touching, n, TPB, s, V, n, cq, ct, bad);
}
void launch_diff3(int n3, const double* a, const double* b, double* out, hipStream_t s) {
  LAUNCH(k_diff3, n3, TPB, s, n3, a, b, out);
}
void launch_tets_positive(const View& V, const double* x, int* bad, hipStream_t s) {
  LAUNCH(k_tets_positive, V.Nt, TPB, s, V, x, bad);
}
void launch_cmap(const View& V, const double* src, double* out, hipStream_t s) {
  LAUNCH(k_cmap, V.Ncv, TPB, s, V, src, out);
}
void launch_cpos(const View& V, hipStream_t s) { LAUNCH(k_cmap, V.Ncv, TPB, s, V, V.x, V.cpos); }
void launch_cdisp(const View& V, const double* p, hipStream_t s) {
  LAUNCH(k_cmap, V.Ncv, TPB, s, V, p, V.cdisp);
}
void launch_cend(const View& V, double* cend, hipStream_t s) {
  LAUNCH(k_cend, 3 * V.Ncv, TPB, s, V, cend);
}
void launch_snap_disp(const View& V, const int* cand, hipStream_t s) {
  LAUNCH(k_snap_disp, V.Ncv, TPB, s, V, cand);
}
void launch_body_resid(const View& V, unsigned long long* res, hipStream_t s) {
  LAUNCH(k_body_resid, V.Ncv, TPB, s, V, res);
}
void launch_bp_targets(const View& V, const double* P0, const double* P1, BroadPhase& bp, int all,
                       hipStream_t s) {
  LAUNCH(k_bp_targets, bp.ntarget, TPB, s, V, P0, P1, bp, all);
}
void launch_bp_count(const View& V, BroadPhase& bp, hipStream_t s) {
  LAUNCH(k_bp_count, bp.ntarget, TPB, s, V, bp);
}
void launch_bp_fill(const View& V, BroadPhase& bp, hipStream_t s) {
  LAUNCH(k_bp_fill, bp.ntarget, TPB, s, V, bp);
}
void launch_bp_query(const View& V, const double* P0, const double* P1, BroadPhase& bp, int all,
                     int emit, int* cand_q, int* cand_t, int* tmp_t, hipStream_t s) {
  const int nb = nblk(V.Nq, TPB / kQueryLanes);
  if (nb > 0)
    hipLaunchKernelGGL(k_bp_query, dim3(nb), dim3(TPB), 0, s, V, P0, P1, bp, all, emit, cand_q,
                       emit ? tmp_t : cand_t);
  if (emit && nb > 0) hipLaunchKernelGGL(k_bp_sort_queries, dim3(nb), dim3(TPB), 0, s, V, bp, tmp_t, cand_t);
}
void launch_narrow(const View& V, int n, const int* cq, const int* ct, int* flag, hipStream_t s) {
  LAUNCH(k_narrow, n, TPB, s, V, n, cq, ct, flag);
}
void launch_compact_pairs(const View& V, int n, const int* cq, const int* ct, const int* flag,
                          const int* pos, int* pkind, int* pv, double* pmeps, int* pscene,
                          hipStream_t s) {
  LAUNCH(k_compact_pairs, n, TPB, s, V, n, cq, ct, flag, pos, pkind, pv, pmeps, pscene);
}
void launch_contact_records(const View& V, int n, const int* cq, const int* ct, const int* flag,
                            const int* pos, int* out, hipStream_t s) {
  LAUNCH(k_contact_records, n, TPB, s, V, n, cq, ct, flag, pos, out);
}
void launch_gather3(int n, const int* idx, const double* src, double* out, hipStream_t s) {
  LAUNCH(k_gather3, n, TPB, s, n, idx, src, out);
}
void launch_body_public(int nb, const double* y, const double* com0, double* out, hipStream_t s) {
  LAUNCH(k_body_public, nb, 64, s, nb, y, com0, out);
}
void launch_count_scene(int n, const int* pscene, int* cnt, hipStream_t s) {
  LAUNCH(k_count_scene, n, TPB, s, n, pscene, cnt);
}
void launch_fem_rows(const View& V, double* g, int mixed, hipStream_t s) {
  const int nb = (V.Nn + kFemRows - 1) / kFemRows;
  if (nb <= 0) return;
  if (mixed) hipLaunchKernelGGL(k_fem_rows<float>, dim3(nb), dim3(kFemRowLanes * kFemRows), 0, s, V, g);
  else hipLaunchKernelGGL(k_fem_rows<double>, dim3(nb), dim3(kFemRowLanes * kFemRows), 0, s, V, g);
}
void launch_barrier_hess(const View& V, int np, const int* pkind, const int* pv,
                         const double* pmeps, double* pg, double* ph, hipStream_t s) {
  if (np > 0) hipLaunchKernelGGL(k_barrier_hess, dim3(np), dim3(64), 0, s, V, np, pkind, pv, pmeps, pg, ph);
}
void launch_body_hess(const View& V, hipStream_t s) { LAUNCH(k_body_hess, V.Nb, 64, s, V); }
void launch_contrib_count(const View& V, int np, const int* pv, int* hcnt, int* gcnt,
                          hipStream_t s) {
  LAUNCH(k_contrib_count, np + V.Nb, TPB, s, V, np, pv, hcnt, gcnt);
}
void launch_contrib_emit(const View& V, int np, const int* pv, const int* hoff, const int* goff,
                         uint64_t* hkey, int* hidx, int* hsrc, double* hcoef, uint64_t* gkey,
                         int* gidx, int* gsrc, double* gcoef, hipStream_t s) {
  LAUNCH(k_contrib_emit, np + V.Nb, TPB, s, V, np, pv, hoff, goff, hkey, hidx, hsrc, hcoef, gkey,
         gidx, gsrc, gcoef);
}
void launch_seg_flags(int n, const uint64_t* keys, int* flags, hipStream_t s) {
  LAUNCH(k_seg_flags, n, TPB, s, n, keys, flags);
}
void launch_seg_start(int n, const int* flags, const int* segid, int* segstart, hipStream_t s) {
  LAUNCH(k_seg_start, n, TPB, s, n, flags, segid, segstart);
}
void launch_reduce_blocks(const View& V, int nmax, const int* nseg, const uint64_t* keys, const int* idx,
                          const int* segstart, const int* src, const double* coef,
                          const double* ph, int* drow, int* dcol, void* dval, int* rowcnt,
                          int mixed, hipStream_t s) {
  if (mixed)
    LAUNCH(k_reduce_blocks<float>, nmax, TPB, s, V, nmax, nseg, keys, idx, segstart, src, coef, ph, drow,
           dcol, static_cast<float*>(dval), rowcnt);
  else
    LAUNCH(k_reduce_blocks<double>, nmax, TPB, s, V, nmax, nseg, keys, idx, segstart, src, coef, ph, drow,
           dcol, static_cast<double*>(dval), rowcnt);
}
void launch_reduce_grad(const View& V, int nmax, const int* nseg, const uint64_t* keys, const int* idx,
                        const int* segstart, const int* src, const double* coef,
                        const double* pg, double* g, hipStream_t s) {
  LAUNCH(k_reduce_grad, nmax, TPB, s, V, nmax, nseg, keys, idx, segstart, src, coef, pg, g);
}
void launch_precond(const View& V, const int* drowptr, const int* dcol, const void* dval,
                    void* pinv, int* bad, int mixed, hipStream_t s) {
  if (mixed) {
    LAUNCH(k_precond_soft<float>, V.Nn, TPB, s, V, drowptr, dcol, static_cast<const float*>(dval),
           static_cast<float*>(pinv), bad);
    if (V.Nb > 0)
      hipLaunchKernelGGL(k_precond_body<float>, dim3(V.Nb), dim3(64), 0, s, V, drowptr, dcol,
                         static_cast<const float*>(dval), bad);
  } else {
    LAUNCH(k_precond_soft<double>, V.Nn, TPB, s, V, drowptr, dcol, static_cast<const double*>(dval),
           static_cast<double*>(pinv), bad);
    if (V.Nb > 0)
      hipLaunchKernelGGL(k_precond_body<double>, dim3(V.Nb), dim3(64), 0, s, V, drowptr, dcol,
                         static_cast<const double*>(dval), bad);
  }
}
template <class T>
void launch_pcg_init(const View& V, const BlockTable& TN, const PcgBufsT<T>& B, hipStream_t s) {
  if (TN.nblk > 0) hipLaunchKernelGGL(k_pcg_init<T>, dim3(xcd_grid(TN.nblk)), dim3(kWave), 0, s, V, TN, B);
}
template <class T>
void launch_pcg_spmv(const View& V, const BlockTable& TN, const BlockTable& TS, const PcgBufsT<T>& B,
                     int parity, hipStream_t s) {
  if (TS.nblk > 0)
    hipLaunchKernelGGL(k_pcg_dir_spmv<T>, dim3(xcd_grid(TS.nblk)), dim3(TPB), 0, s, V, TN, TS, B, parity);
}
template <class T>
void launch_pcg_update(const View& V, const BlockTable& TN, const BlockTable& TS, const PcgBufsT<T>& B,
                       int parity, hipStream_t s) {
  if (TN.nblk <= 0) return;
  if (B.cg_mmax <= kWave)
    hipLaunchKernelGGL((k_pcg_update<T, kWave>), dim3(xcd_grid(TN.nblk)), dim3(kWave), 0, s, V, TN, TS, B, parity);
  else
    hipLaunchKernelGGL((k_pcg_update<T, TPB>), dim3(xcd_grid(TN.nblk)), dim3(TPB), 0, s, V, TN, TS, B, parity);
}
template <class T>
void launch_pcg_coarse(const View& V, const BlockTable& TN, const PcgBufsT<T>& B, T* prz, hipStream_t s) {
  if (TN.nblk > 0 && B.cg_on) hipLaunchKernelGGL(k_pcg_coarse<T>, dim3(xcd_grid(TN.nblk)), dim3(kWave), 0, s, V, TN, B, prz);
}
template void launch_pcg_coarse<double>(const View&, const BlockTable&, const PcgBufsT<double>&, double*, hipStream_t);
template void launch_pcg_coarse<float>(const View&, const BlockTable&, const PcgBufsT<float>&, float*, hipStream_t);
template void launch_pcg_init<double>(const View&, const BlockTable&, const PcgBufsT<double>&, hipStream_t);
template void launch_pcg_init<float>(const View&, const BlockTable&, const PcgBufsT<float>&, hipStream_t);
template void launch_pcg_spmv<double>(const View&, const BlockTable&, const BlockTable&, const PcgBufsT<double>&, int, hipStream_t);
template void launch_pcg_spmv<float>(const View&, const BlockTable&, const BlockTable&, const PcgBufsT<float>&, int, hipStream_t);
template void launch_pcg_update<double>(const View&, const BlockTable&, const BlockTable&, const PcgBufsT<double>&, int, hipStream_t);
template void launch_pcg_update<float>(const View&, const BlockTable&, const BlockTable&, const PcgBufsT<float>&, int, hipStream_t);
void launch_pmax(const View& V, const double* p, unsigned long long* pmax, hipStream_t s) {
  LAUNCH(k_pmax, V.Nn + V.Ncv, TPB, s, V, p, pmax);
}
void launch_to_f32(size_t n, const double* src, float* dst, hipStream_t s) {
  if (n == 0) return;
  const size_t nb = std::min<size_t>((n + TPB - 1) / TPB, 65536);
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)nb), dim3(TPB), 0, s, n, src, dst);
}
void launch_refine_resid(const View& V, const BlockTable& TS, const int* drowptr, const int* dcol,
                         const double* dval, const double* g, const double* dx, double* gres,
                         hipStream_t s) {
  if (TS.nblk > 0)
    hipLaunchKernelGGL(k_refine_resid, dim3(xcd_grid(TS.nblk)), dim3(TPB), 0, s, V, TS, drowptr, dcol,
                       dval, g, dx, gres);
}
void launch_refine_norm(const View& V, const BlockTable& TN, const double* pinv, const double* g,
                        const double* gres, double* part, hipStream_t s) {
  if (TN.nblk > 0)
    hipLaunchKernelGGL(k_refine_norm, dim3(xcd_grid(TN.nblk)), dim3(kWave), 0, s, V, TN, pinv, g, gres, part);
}
void launch_refine_apply(const View& V, const double* c, double* dx, int assign, hipStream_t s) {
  LAUNCH(k_refine_apply, 3 * V.Nn, TPB, s, V, c, dx, assign);
}
void launch_ccd(const View& V, int n, const int* cq, const int* ct, unsigned long long* amin,
                hipStream_t s) {
  LAUNCH(k_ccd, n, 64, s, V, n, cq, ct, amin);
}
void launch_scene_offsets(const View& V, int n, const int* cq, int* off, hipStream_t s) {
  LAUNCH(k_scene_offsets, n + 1, TPB, s, V, n, cq, off);
}
void launch_line_search(const View& V, const BlockTable& TN, const BlockTable& TT, const BlockTable& TP,
                        int ncand, const int* cq, const int* ct, const LsBufs& L, hipStream_t s) {
  if (TN.nblk > 0) hipLaunchKernelGGL(k_ls_nodes, dim3(TN.nblk), dim3(kWave), 0, s, V, TN, L);
  if (TT.nblk > 0) hipLaunchKernelGGL(k_ls_tets, dim3(TT.nblk), dim3(TPB), 0, s, V, TT, L);
  LAUNCH(k_ls_bodies, kLsSlots * V.Nb, 64, s, V, L);
  LAUNCH(k_ls_pairs, kLsSlots * ncand, 64, s, V, ncand, cq, ct, L);
  if (TP.nblk > 0) hipLaunchKernelGGL(k_ls_pair_sums, dim3(TP.nblk), dim3(TPB), 0, s, V, TP, L);
  LAUNCH(k_ls_fric, kLsSlots * L.F.n, 64, s, V, L);
  hipLaunchKernelGGL(k_ls_reduce, dim3(V.S), dim3(TPB), 0, s, V, TN, TT, TP, L);
}
void launch_update(const View& V, const double* p, const double* alpha, hipStream_t s) {
  LAUNCH(k_update, V.Nn, TPB, s, V, p, alpha);
}
void launch_al_apply(const View& V, const int* action, hipStream_t s) {
  LAUNCH(k_al_apply, V.Nb, 64, s, V, action);
}
void launch_body_reset(const View& V, double kappa0, hipStream_t s) {
  LAUNCH(k_body_reset, V.Nb, 64, s, V, kappa0);
}
void launch_body_clear_lambda(const View& V, const int* flag, hipStream_t s) {
  LAUNCH(k_body_clear_lambda, V.Nb, 64, s, V, flag);
}
void launch_velocity(const View& V, const int* ok, hipStream_t s) {
  LAUNCH(k_velocity, V.Nn, TPB, s, V, ok);
}
void launch_rollback(const View& V, const int* failed, hipStream_t s) {
  LAUNCH(k_rollback, V.Nn, TPB, s, V, failed);
}
void launch_debug_fem(int n, const double* x, const double* Dminv, const double* vol, double mu,
                      double lam, double* e, double* g, double* H, double* Hp, hipStream_t s) {
  LAUNCH(k_debug_fem, n, 64, s, n, x, Dminv, vol, mu, lam, e, g, H, Hp);
}
void launch_debug_barrier(int n, const int* kinds, const double* x, const double* meps,
                          double dhat, double kappa, double* e, double* g, double* H, double* Hp,
                          int* types, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_debug_barrier, dim3(n), dim3(64), 0, s, n, kinds, x, meps, dhat, kappa, e, g, H, Hp, types);
}
void launch_fric_build(const View& V, int n, const int* pkind, const int* pv, const double* pmeps,
                       const FricBufs& F, hipStream_t s) {
  LAUNCH(k_fric_build, n, 64, s, V, n, pkind, pv, pmeps, F);
}
void launch_fric_derivs(const View& V, const FricBufs& F, int off, int* pv, double* pg, double* ph,
                        hipStream_t s) {
  LAUNCH(k_fric_derivs, F.n, 64, s, V, F, off, pv, pg, ph);
}
void launch_debug_friction(int n, const int* kinds, const double* xn, const double* x,
                           const double* meps, double dhat, double kappa, double mu, double eh,
                           double* lam, double* e, double* g, double* H, hipStream_t s) {
  LAUNCH(k_debug_friction, n, 64, s, n, kinds, xn, x, meps, dhat, kappa, mu, eh, lam, e, g, H);
}
void launch_debug_ccd(int n, const int* kinds, const double* x, const double* p, double gap,
                      int max_iter, double* t, hipStream_t s) {
  LAUNCH(k_debug_ccd, n, 64, s, n, kinds, x, p, gap, max_iter, t);
}
void launch_debug_arap(int n, const double* A, double* e, double* g, double* H, double* Hp,
                       hipStream_t s) {
  LAUNCH(k_debug_arap, n, 64, s, n, A, e, g, H, Hp);
}

}  // namespace tc
