"""Host logic of the two-level preconditioner (coarse.h), no GPU: the inverse coarse operator
it forms must invert P^T K P, with P the rigid modes of each aggregate and K the rest-state
Newton matrix assembled independently from the oracle's neo-Hookean tet Hessians."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2504_12908_amd import scenes as S

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2504_12908_amd", "csrc")
MU = S.GEL_E / (2 * (1 + S.GEL_NU))
LAM = S.GEL_E * S.GEL_NU / ((1 + S.GEL_NU) * (1 - 2 * S.GEL_NU))


@pytest.fixture(scope="module")
def coarse_lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("coarse") / "libcoarse.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-I", CSRC, "-o", out,
                    os.path.join(HERE, "host", "coarse_wrap.cpp")], check=True)
    return C.CDLL(out)


def _morton_perm(V):
    lo, hi = V.min(0), V.max(0)
    q = np.minimum(1023, np.floor((V - lo) / np.where(hi > lo, hi - lo, 1) * 1024)).astype(np.int64)
    key = np.zeros(len(V), np.int64)
    for b in range(9, -1, -1):
        for c in (2, 1, 0):
            key = (key << 1) | ((q[:, c] >> b) & 1)
    order = np.lexsort((np.arange(len(V)), key))
    perm = np.empty(len(V), int)
    perm[order] = np.arange(len(V))
    return perm


def _run(lib, spec, max_agg):
    h = spec.params["h"]
    nv, nt = len(spec.verts), len(spec.tets)
    perm = _morton_perm(spec.verts)
    V = np.empty_like(spec.verts)
    V[perm] = spec.verts
    T = perm[spec.tets].astype(np.int32)
    dirich = np.empty(nv, np.uint8)
    dirich[perm] = spec.dirichlet
    nfree = (dirich == 0).astype(np.int32)
    Dm = np.stack([V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]], V[T[:, 3]] - V[T[:, 0]]], axis=2)
    Dminv = np.ascontiguousarray(np.linalg.inv(Dm).reshape(nt, 9))
    vol = np.linalg.det(Dm) / 6
    mass = np.zeros(nv)
    np.add.at(mass, T.ravel(), np.repeat(S.GEL_RHO * vol / 4, 4))
    nblk = ((nv + 3) // 4 * 4 + 63) // 64
    tn_b0 = (np.arange(nblk) * 64).astype(np.int32)
    ba = np.zeros(nblk, np.int32)
    nagg = C.c_int()
    ab0, ab1 = np.zeros(nblk, np.int32), np.zeros(nblk, np.int32)
    d = np.zeros(3 * nv)
    ainv = np.zeros((6 * nblk) ** 2)
    ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int))
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    m = lib.coarse_build(nv, ip(nfree), dp(np.ascontiguousarray(V)), dp(mass), nt,
                         ip(np.ascontiguousarray(T)), dp(Dminv), dp(vol), C.c_double(h),
                         C.c_double(MU), C.c_double(LAM), nblk, ip(tn_b0), max_agg, ip(ba),
                         C.byref(nagg), ip(ab0), ip(ab1), dp(d), dp(ainv))
    return dict(V=V, T=T, nfree=nfree, mass=mass, h=h, m=m, nagg=nagg.value, blk_agg=ba,
                agg_b0=ab0[:nagg.value], agg_b1=ab1[:nagg.value], d=d.reshape(nv, 3),
                Ainv=ainv[:m * m].reshape(m, m))


def _independent(oracle_lib, r):
    V, T, free = r["V"], r["T"], r["nfree"].astype(bool)
    node = -np.ones(len(V), int)
    node[free] = np.arange(free.sum())
    nf = int(free.sum())
    rows, cols, vals = [], [], []
    for e in range(len(T)):
        x = V[T[e]]
        _, _, _, Hp = oracle_lib.nh_tet(x, x, MU, LAM)
        for a in range(4):
            for b in range(4):
                na, nb = node[T[e, a]], node[T[e, b]]
                if na < 0 or nb < 0:
                    continue
                for c in range(3):
                    for dd in range(3):
                        rows.append(3 * na + c)
                        cols.append(3 * nb + dd)
                        vals.append(r["h"] ** 2 * Hp[3 * a + c, 3 * b + dd])
    for i in np.nonzero(free)[0]:
        for c in range(3):
            rows.append(3 * node[i] + c)
            cols.append(3 * node[i] + c)
            vals.append(r["mass"][i])
    K = sp.csr_matrix((vals, (rows, cols)), shape=(3 * nf, 3 * nf))
    m = r["m"]
    P = np.zeros((3 * nf, m))
    for i in np.nonzero(free)[0]:
        a = r["blk_agg"][i // 64]
        for c in range(3):
            P[3 * node[i] + c, 6 * a + c] = 1.0
        for k in range(3):
            e = np.zeros(3)
            e[k] = 1.0
            P[3 * node[i]:3 * node[i] + 3, 6 * a + 3 + k] = np.cross(e, r["d"][i])
    return P, K


@pytest.mark.parametrize("max_agg", [128, 2])
def test_coarse_inverse_matches_independent_assembly(coarse_lib, oracle_lib, max_agg):
    spec = S.pad_press_cube(0)
    r = _run(coarse_lib, spec, max_agg)
    nblk = len(r["blk_agg"])
    assert r["nagg"] == (nblk if max_agg >= nblk else (nblk + 1) // 2)
    P, K = _independent(oracle_lib, r)
    Ac = P.T @ (K @ P)
    Ai = r["Ainv"]
    assert np.array_equal(Ai, Ai.T)
    # modes of aggregates without free nodes are dropped (zero rows); the rest is inverted
    kept = np.abs(Ai).sum(axis=1) > 0
    R = Ai @ Ac
    assert np.abs(R[np.ix_(kept, kept)] - np.eye(kept.sum())).max() < 1e-9
    assert np.all(np.abs(Ac[~kept]).max(initial=0.0) < 1e-12 * np.abs(Ac).max())
    # every aggregate with at least 3 non-collinear free nodes keeps all 6 modes
    free = r["nfree"].astype(bool)
    for a in range(r["nagg"]):
        nodes = [i for i in range(len(free)) if free[i] and r["blk_agg"][i // 64] == a]
        if len(nodes) >= 4:
            assert kept[6 * a:6 * a + 6].all()
    # offsets are centred per aggregate and scaled to unit RMS radius
    for a in range(r["nagg"]):
        nodes = [i for i in range(len(free)) if free[i] and r["blk_agg"][i // 64] == a]
        if nodes:
            dd = r["d"][nodes]
            assert np.abs(dd.mean(axis=0)).max() < 1e-12
            assert abs(np.sqrt((dd ** 2).sum(axis=1).mean()) - 1.0) < 1e-12
