"""CPU oracle for the UAV coverage-path QUBO annealer -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does.

Thin ctypes wrapper over ``oracle.c`` (plain C, built by ``oracle/build.py``).
Every function documents the passage of the paper it follows; the readings
taken where the paper is silent are listed in the C file's comments.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build(force=True)
        L = C.CDLL(_build.LIB)
        P = C.POINTER
        i32, i64, u32, u64, u8, dbl = C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_uint8, C.c_double
        L.orc_philox4x32_10.argtypes = [P(u32), P(u32), P(u32)]
        L.orc_accept_word.argtypes = [u32, u32, u32, u32, C.c_int, C.c_int]
        L.orc_accept_word.restype = u32
        L.orc_init_bit.argtypes = [u32, u32, u32, C.c_int, C.c_int]
        L.orc_init_bit.restype = u32
        L.orc_cost.argtypes = [i32, i32, i32, i32]
        L.orc_cost.restype = i32
        L.orc_free_cells.argtypes = [i32, i32, i32, P(u8), P(i32)]
        L.orc_free_cells.restype = i32
        L.orc_cost_matrix.argtypes = [i32, i32, i32, P(i32), i32, P(i32)]
        L.orc_cost_matrix.restype = i32
        L.orc_literal_energy.argtypes = [i32, P(i32), i32, i32, P(u8)]
        L.orc_literal_energy.restype = i64
        L.orc_J.argtypes = [i32, P(i32), i32, i32, i32]
        L.orc_J.restype = i32
        L.orc_build_qubo.argtypes = [i32, P(i32), i32, i32, P(i32), P(i32), P(i64)]
        L.orc_qubo_energy.argtypes = [i32, P(i32), P(i32), i64, P(u8)]
        L.orc_qubo_energy.restype = i64
        L.orc_temperature.argtypes = [dbl, dbl, i32, i32]
        L.orc_temperature.restype = dbl
        L.orc_dmax.argtypes = [dbl]
        L.orc_dmax.restype = i32
        L.orc_thresholds.argtypes = [dbl, dbl, i32, i32, P(u32)]
        L.orc_anneal.argtypes = [i32, P(i32), P(i32), i32, P(i32), i64, i32, i32, P(u32), u32, u32, i32, P(i32),
                                 P(u8), P(i32), i32, P(u8), P(i64), P(i64), P(i32), P(u8), P(u64),
                                 P(u64), P(i64), i32]
        L.orc_anneal.restype = i32
        L.orc_enum_min.argtypes = [i32, P(i32), P(i32), i64, P(i64), P(i64), P(u8), P(i64)]
        L.orc_enum_min.restype = i32
        L.orc_tour_brute.argtypes = [i32, P(i32), i32, P(i64), P(i64)]
        L.orc_tour_brute.restype = i32
        L.orc_held_karp.argtypes = [i32, P(i32), i32]
        L.orc_held_karp.restype = i64
        L.orc_pt_temperature.argtypes = [dbl, dbl, i32, i32]
        L.orc_pt_temperature.restype = dbl
        L.orc_pt_dx.argtypes = [dbl, dbl, i32, i32, P(i32)]
        L.orc_pt_dx.restype = i32
        L.orc_pt_tables.argtypes = [dbl, dbl, i32, P(i32), i32, P(u32)]
        L.orc_pt_word.argtypes = [u32, u32, u32, u32, i32]
        L.orc_pt_word.restype = u32
        L.orc_pt_exchange.argtypes = [i32, i32, i32, u32, u32, u32, P(i32), i32, P(u32), P(u8), P(i64), P(u64)]
        L.orc_pt_exchange.restype = i32
        L.orc_pt_anneal.argtypes = [i32, P(i32), P(i32), i32, P(i32), i64, i32, i32, i32, i32, P(u32), P(i32), i32,
                                    P(u32), u32, u32, i32, P(i32), P(u8), P(i64), P(i64), P(i32), P(u8), P(u64),
                                    P(u64), P(u64), i32]
        L.orc_pt_anneal.restype = i32
        _lib = L
    return _lib


def _p(a, ct):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ct))


# --------------------------------------------------------------------------
# Philox4x32-10 (Salmon et al., SC'11)
# --------------------------------------------------------------------------
def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


def accept_word(seed, inst, r, s, t, c):
    return int(lib().orc_accept_word(seed, inst, r, s, t, c))


def init_bit(seed, inst, r, t, c):
    return int(lib().orc_init_bit(seed, inst, r, t, c))


# --------------------------------------------------------------------------
# Instance + QUBO (Sec. II system model; Sec. III-B eqs. (3)-(6))
# --------------------------------------------------------------------------
def cost(cols, ga, gb, scale=10):
    return int(lib().orc_cost(cols, ga, gb, scale))


class OracleQubo:
    """The oracle's own view of one instance: free cells, cost matrix over
    [depot] + F, penalty, and the expanded QUBO (c0, b, dense J)."""

    def __init__(self, rows, cols, nofly=None, depot=0, scale=10, penalty=0, closed=True, dense=True):
        self.rows, self.cols, self.depot, self.scale, self.closed = rows, cols, depot, scale, bool(closed)
        nf = None
        if nofly is not None:
            nf = np.ascontiguousarray(nofly, dtype=np.uint8).reshape(-1)
            assert nf.size == rows * cols
        self.nofly = nf
        L = lib()
        m = L.orc_free_cells(rows, cols, depot, _p(nf, C.c_uint8), None)
        self.m, self.N = m, m * m
        self.F = np.zeros(max(m, 1), np.int32)[:m].copy()
        L.orc_free_cells(rows, cols, depot, _p(nf, C.c_uint8), _p(self.F, C.c_int32))
        self.W = np.zeros((m + 1, m + 1), np.int32)
        self.wmax = int(L.orc_cost_matrix(cols, depot, m, _p(self.F, C.c_int32), scale, _p(self.W, C.c_int32)))
        self.P = int(penalty) if penalty else 2 * self.wmax
        self.b = np.zeros(self.N, np.int32)
        self.J = np.zeros((self.N, self.N), np.int32) if dense else None
        c0 = C.c_int64(0)
        L.orc_build_qubo(m, _p(self.W, C.c_int32), self.P, int(self.closed), _p(self.J, C.c_int32),
                         _p(self.b, C.c_int32), C.byref(c0))
        self.c0 = int(c0.value)

    def J_entry(self, k, l):
        return int(lib().orc_J(self.m, _p(self.W, C.c_int32), self.P, k, l))

    def literal_energy(self, x):
        x = np.ascontiguousarray(x, dtype=np.uint8).reshape(-1)
        assert x.size == self.N
        return int(lib().orc_literal_energy(self.m, _p(self.W, C.c_int32), self.P, int(self.closed),
                                            _p(x, C.c_uint8)))

    def energy(self, x):
        assert self.J is not None
        x = np.ascontiguousarray(x, dtype=np.uint8).reshape(-1)
        return int(lib().orc_qubo_energy(self.N, _p(self.J, C.c_int32), _p(self.b, C.c_int32), self.c0,
                                         _p(x, C.c_uint8)))

    def tour_brute(self):
        best, n = C.c_int64(0), C.c_int64(0)
        rc = lib().orc_tour_brute(self.m, _p(self.W, C.c_int32), int(self.closed), C.byref(best), C.byref(n))
        assert rc == 0
        return int(best.value), int(n.value)

    def held_karp(self):
        return int(lib().orc_held_karp(self.m, _p(self.W, C.c_int32), int(self.closed)))

    def enum_min(self):
        assert self.J is not None and self.N <= 24
        mn, cnt, inf = C.c_int64(0), C.c_int64(0), C.c_int64(0)
        arg = np.zeros(max(self.N, 1), np.uint8)
        rc = lib().orc_enum_min(self.m, _p(self.J, C.c_int32), _p(self.b, C.c_int32), self.c0, C.byref(mn),
                                C.byref(cnt), _p(arg, C.c_uint8), C.byref(inf))
        assert rc == 0
        return int(mn.value), int(cnt.value), arg[: self.N], int(inf.value)

    def decode(self, x):
        """Visiting order (grid indices) of a permutation state, or None."""
        X = np.asarray(x, dtype=np.uint8).reshape(self.m, self.m)
        if not ((X.sum(0) == 1).all() and (X.sum(1) == 1).all()):
            return None
        order = [int(self.F[int(np.argmax(X[t]))]) for t in range(self.m)]
        return [self.depot] + order + ([self.depot] if self.closed else [])

    def path_cost(self, path):
        return sum(cost(self.cols, a, b, self.scale) for a, b in zip(path[:-1], path[1:]))


# --------------------------------------------------------------------------
# Schedule + thresholds
# --------------------------------------------------------------------------
def temperature(T0, T1, S, s):
    return float(lib().orc_temperature(T0, T1, S, s))


def thresholds(T0, T1, S):
    L = lib()
    dmax = int(L.orc_dmax(T0))
    thr = np.zeros((S, dmax + 1), np.uint32)
    L.orc_thresholds(T0, T1, S, dmax, _p(thr, C.c_uint32))
    return dmax, thr


# --------------------------------------------------------------------------
# Annealer
# --------------------------------------------------------------------------
def anneal(q, sweeps, T0, T1, seed, inst, replicas, init_x=None, start_sweep=None, check_every=0,
           threads=0, table=None):
    """Run replicas ``replicas`` (list of replica ids) of instance id ``inst``.

    Uses the stored J when the instance has one, otherwise evaluates every
    coefficient from its definition where it is needed (large fields).
    Returns a dict of numpy arrays indexed like ``replicas``."""
    reps = np.ascontiguousarray(replicas, dtype=np.int32)
    n = reps.size
    N = q.N
    dmax, thr = table if table is not None else thresholds(T0, T1, sweeps)
    assert thr.shape == (sweeps, dmax + 1)
    ix = None
    if init_x is not None:
        ix = np.ascontiguousarray(init_x, dtype=np.uint8).reshape(n, N)
    ss = None
    if start_sweep is not None:
        ss = np.ascontiguousarray(np.broadcast_to(np.asarray(start_sweep, np.int32), (n,)), dtype=np.int32)
    out = dict(
        final_x=np.zeros((n, N), np.uint8), final_E=np.zeros(n, np.int64), best_E=np.zeros(n, np.int64),
        best_sweep=np.zeros(n, np.int32), best_x=np.zeros((n, N), np.uint8), accepts=np.zeros(n, np.uint64),
        draws=np.zeros(n, np.uint64), mismatches=np.zeros(n, np.int64))
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    rc = lib().orc_anneal(
        q.m, _p(q.J, C.c_int32), _p(q.W, C.c_int32), q.P, _p(q.b, C.c_int32), q.c0, sweeps, dmax,
        _p(thr, C.c_uint32),
        seed, inst, n, _p(reps, C.c_int32), _p(ix, C.c_uint8), _p(ss, C.c_int32), check_every,
        _p(out["final_x"], C.c_uint8), _p(out["final_E"], C.c_int64), _p(out["best_E"], C.c_int64),
        _p(out["best_sweep"], C.c_int32), _p(out["best_x"], C.c_uint8), _p(out["accepts"], C.c_uint64),
        _p(out["draws"], C.c_uint64), _p(out["mismatches"], C.c_int64), threads)
    assert rc == 0
    return out


def instance_best(res, replicas):
    """Per-instance result: lexicographic minimum of (best_E, replica id)."""
    reps = np.asarray(replicas)
    order = np.lexsort((reps, res["best_E"]))
    i = int(order[0])
    return dict(best_E=int(res["best_E"][i]), best_replica=int(reps[i]), best_sweep=int(res["best_sweep"][i]),
                best_x=res["best_x"][i].copy())


# --------------------------------------------------------------------------
# Replica exchange (parallel tempering): K chains per replica index at the
# fixed temperatures of a geometric ladder, neighbouring slots trading states
# by the Metropolis rule on the product of their Boltzmann weights.  An
# extension of the many-replica search of Sec. III-C; the rule and the draw
# addressing are stated in oracle.c.
# --------------------------------------------------------------------------
PT_DX_CAP = 1 << 22


def pt_ladder(T_hot, T_cold, K):
    """(T[K], DX[K-1], xthr[K-1][stride]) of the ladder."""
    T = np.array([lib().orc_pt_temperature(T_hot, T_cold, K, k) for k in range(K)])
    DX = np.zeros(max(K - 1, 1), np.int32)
    mx = lib().orc_pt_dx(T_hot, T_cold, K, PT_DX_CAP, _p(DX, C.c_int32)) if K > 1 else 1
    if mx < 0:
        raise ValueError("ladder needs T_cold < T_hot and exchange tables within the cap")
    stride = mx + 1
    xthr = np.zeros((max(K - 1, 1), stride), np.uint32)
    if K > 1:
        lib().orc_pt_tables(T_hot, T_cold, K, _p(DX, C.c_int32), stride, _p(xthr, C.c_uint32))
    return T, DX[:K - 1].copy(), xthr[:K - 1].copy()


def pt_exchange(x, E, rnd, seed, inst, DX, xthr, swaps=None):
    """One exchange round in place.  x: uint8 [K, R, N]; E: int64 [K, R]."""
    K, R, N = x.shape
    assert x.flags.c_contiguous and E.flags.c_contiguous and E.shape == (K, R)
    sw = swaps if swaps is not None else np.zeros(max(K - 1, 1), np.uint64)
    xthr = np.ascontiguousarray(xthr, dtype=np.uint32)
    lib().orc_pt_exchange(K, R, N, rnd, seed, inst, _p(np.ascontiguousarray(DX, np.int32), C.c_int32),
                          xthr.shape[1] if K > 1 else 1, _p(xthr, C.c_uint32), _p(x, C.c_uint8),
                          _p(E, C.c_int64), _p(sw, C.c_uint64))
    return sw


def pt_anneal(q, K, R, sweeps, T_hot, T_cold, seed, inst, interval=1, threads=0):
    """Parallel tempering: slot k (instance id inst + k, constant temperature
    T_k) sweeps chains 0..R-1 like ``anneal``; after every ``interval`` sweeps,
    unless the schedule has ended or K = 1, exchange round e = 0, 1, ... runs
    (its draws addressed by ``inst``).  Each slot keeps its
    own best (the strict minimum over its sweep ends) and counters."""
    T, DX, xthr = pt_ladder(T_hot, T_cold, K)
    N = q.N
    reps = list(range(R))
    x = np.zeros((K, R, N), np.uint8)
    E = np.zeros((K, R), np.int64)
    best_E = np.full((K, R), np.iinfo(np.int64).max, np.int64)
    best_sweep = np.full((K, R), -1, np.int32)
    best_x = np.zeros((K, R, N), np.uint8)
    acc = np.zeros((K, R), np.uint64)
    drw = np.zeros((K, R), np.uint64)
    swaps = np.zeros(max(K - 1, 1), np.uint64)
    tables = [thresholds(T[k], T[k], sweeps) for k in range(K)]
    b, e = 0, 0
    while b < sweeps:
        end = min(b + interval, sweeps)
        for k in range(K):
            dmax, thr = tables[k]
            res = anneal(q, end, T[k], T[k], seed, (inst + k) & 0xFFFFFFFF, reps,
                         init_x=x[k] if b > 0 else None, start_sweep=b if b > 0 else None,
                         threads=threads, table=(dmax, thr[:end].copy()))
            x[k] = res["final_x"]
            E[k] = res["final_E"]
            better = res["best_E"] < best_E[k]
            best_E[k][better] = res["best_E"][better]
            best_sweep[k][better] = res["best_sweep"][better]
            best_x[k][better] = res["best_x"][better]
            acc[k] += res["accepts"]
            drw[k] += res["draws"]
        if end < sweeps and K > 1:
            pt_exchange(x, E, e, seed, inst, DX, xthr, swaps)
            e += 1
        b = end
    return dict(T=T, final_x=x, final_E=E, best_E=best_E, best_sweep=best_sweep, best_x=best_x, accepts=acc,
                draws=drw, swaps=swaps[:K - 1], rounds=e)


def pt_anneal_chains(q, K, chains, sweeps, T_hot, T_cold, seed, inst, interval=1, threads=0):
    """The tempering of ``pt_anneal`` for the listed chain ids only, as one C
    loop per chain that keeps its fields across exchange rounds (chains are
    independent, so any subset gives those chains' outputs).  Arrays are
    indexed [chain index, slot]; swaps per chain and pair."""
    T, DX, xthr = pt_ladder(T_hot, T_cold, K)
    rows = [thresholds(T[k], T[k], 1) for k in range(K)]
    dmax = max(d for d, _ in rows)
    thr = np.zeros((K, dmax + 1), np.uint32)
    for k, (d, t) in enumerate(rows):
        thr[k, :d + 1] = t[0]
    ch = np.ascontiguousarray(chains, dtype=np.int32)
    n, N = ch.size, q.N
    out = dict(final_x=np.zeros((n, K, N), np.uint8), final_E=np.zeros((n, K), np.int64),
               best_E=np.zeros((n, K), np.int64), best_sweep=np.zeros((n, K), np.int32),
               best_x=np.zeros((n, K, N), np.uint8), accepts=np.zeros((n, K), np.uint64),
               draws=np.zeros((n, K), np.uint64), swaps=np.zeros((n, max(K - 1, 1)), np.uint64))
    DXa = np.ascontiguousarray(DX if K > 1 else np.zeros(1, np.int32), dtype=np.int32)
    xt = np.ascontiguousarray(xthr if K > 1 else np.zeros((1, 2), np.uint32), dtype=np.uint32)
    rc = lib().orc_pt_anneal(q.m, _p(q.J, C.c_int32), _p(q.W, C.c_int32), q.P, _p(q.b, C.c_int32), q.c0, K, sweeps,
                             interval, dmax, _p(thr, C.c_uint32), _p(DXa, C.c_int32), xt.shape[1], _p(xt, C.c_uint32),
                             seed, inst, n, _p(ch, C.c_int32), _p(out["final_x"], C.c_uint8),
                             _p(out["final_E"], C.c_int64), _p(out["best_E"], C.c_int64),
                             _p(out["best_sweep"], C.c_int32), _p(out["best_x"], C.c_uint8),
                             _p(out["accepts"], C.c_uint64), _p(out["draws"], C.c_uint64),
                             _p(out["swaps"], C.c_uint64), threads)
    assert rc == 0
    out["swaps"] = out["swaps"][:, :K - 1]
    out["T"] = T
    return out
