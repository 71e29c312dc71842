"""ctypes wrapper of the CPU FP64 oracle (libsidm_oracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark.  The product path never imports it.

All arrays are numpy, halo-local, structure of arrays.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libsidm_oracle.so")
_lib = None

EVENT_DTYPE = np.dtype([("a", np.uint32), ("b", np.uint32), ("ia", np.int64),
                        ("ib", np.int64), ("u", np.float64), ("P", np.float64)],
                       align=True)


class OrcParams(C.Structure):
    _fields_ = [("G", C.c_double), ("eps", C.c_double), ("sigma_m", C.c_double),
                ("dt", C.c_double), ("k", C.c_int32), ("seed", C.c_uint64),
                ("host_kind", C.c_int32), ("host_rho_s", C.c_double),
                ("host_r_s", C.c_double), ("host_c", C.c_double * 3), ("sigma_w", C.c_double),
                ("host_hern_M", C.c_double), ("host_hern_a", C.c_double),
                ("host_disk", (C.c_double * 3) * 4), ("boundary_r", C.c_double),
                ("boundary_c", C.c_double * 3), ("eta", C.c_double), ("dt_min", C.c_double),
                ("max_bin", C.c_int32), ("tree_alpha", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from oracle import build as _b
            _b.build()
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_u32p = C.POINTER(C.c_uint32)
_i64p = C.POINTER(C.c_int64)
_u8p = C.POINTER(C.c_uint8)


def _declare(L):
    L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    L.orc_u53.argtypes = [C.c_uint32, C.c_uint32]
    L.orc_u53.restype = C.c_double
    L.orc_accept_u.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]
    L.orc_accept_u.restype = C.c_double
    L.orc_kernel_W.argtypes = [C.c_double, C.c_double]
    L.orc_kernel_W.restype = C.c_double
    L.orc_lambda.argtypes = [C.c_double, C.c_double, C.c_double]
    L.orc_lambda.restype = C.c_double
    L.orc_gravity.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, C.c_double, C.c_double,
                              C.c_int64, _i64p, _dp, _dp, _dp, _dp, _dp]
    L.orc_tree_gravity.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, C.c_double,
                                   C.c_double, C.c_double, C.c_int64, _i64p, _dp, _dp, _dp, _dp,
                                   _i64p]
    L.orc_octree_gravity.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                     C.c_double, C.c_double, C.c_double, C.c_int64, _i64p, _dp,
                                     _dp, _dp, _dp, _i64p]
    L.orc_host_nfw.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_double, C.c_double,
                               C.c_double, _dp, _dp, _dp, _dp, _dp]
    L.orc_knn.argtypes = [C.c_int64, _dp, _dp, _dp, _u32p, C.c_int32, C.c_int64,
                          _i64p, _dp, _u32p]
    L.orc_sigma.argtypes = [C.c_double, C.c_double, C.c_double]
    L.orc_sigma.restype = C.c_double
    L.orc_find_events.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _u32p,
                                  _dp, C.c_double, C.c_double, C.c_double, C.c_uint64, C.c_uint32,
                                  _u8p, C.c_void_p, C.c_int64, _i64p, _i64p]
    L.orc_find_events.restype = C.c_int64
    L.orc_host_hernquist.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_double, C.c_double,
                                     C.c_double, C.POINTER(C.c_double), _dp, _dp, _dp, _dp]
    L.orc_host_disk.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                C.c_double, C.POINTER(C.c_double), _dp, _dp, _dp, _dp]
    L.orc_host_field.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_void_p, _dp, _dp, _dp, _dp]
    L.orc_bin.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32,
                          C.c_double, C.c_double, C.c_double]
    L.orc_bin.restype = C.c_int32
    L.orc_tidal_radius.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, C.c_void_p, _dp, _dp,
                                   _i64p]
    L.orc_tidal_radius.restype = C.c_int
    L.orc_knn_grid.argtypes = [C.c_int64, _dp, _dp, _dp, _u32p, C.c_int32, _dp]
    L.orc_knn_tree.argtypes = [C.c_int64, _dp, _dp, _dp, _u32p, C.c_int32, _dp, _u32p]
    L.orc_find_events_tree.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _u32p,
                                       _dp, C.c_double, C.c_double, C.c_double, C.c_uint64,
                                       C.c_uint32, C.c_void_p, C.c_int64, _i64p, _i64p]
    L.orc_find_events_tree.restype = C.c_int64
    L.orc_find_events_sweep.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _u32p,
                                        _dp, C.c_double, C.c_double, C.c_double, C.c_uint64,
                                        C.c_uint32,
                                        C.c_void_p, C.c_int64, _i64p, _i64p]
    L.orc_find_events_sweep.restype = C.c_int64
    L.orc_central_density.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, C.c_double, _i64p,
                                      _i64p, _dp]
    L.orc_kick_pair.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                C.c_double, C.c_double, _dp, _dp]
    L.orc_apply_events.argtypes = [C.c_int64, C.c_void_p, _dp, _dp, _dp, _dp,
                                   C.c_uint64, C.c_uint32]
    L.orc_diag.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_kdk_step.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _u32p,
                               _dp, _dp, _dp, _dp, _dp, C.POINTER(OrcParams),
                               C.c_uint32, C.c_void_p, C.c_int64]
    L.orc_kdk_step.restype = C.c_int64
    L.orc_kick_drift.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                 C.POINTER(OrcParams)]
    L.orc_close_kick.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, C.POINTER(OrcParams)]
    L.orc_num_threads.restype = C.c_int
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_set_threads.restype = None


def _d(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads():
    return int(lib().orc_num_threads())


def set_threads(n):
    """Threads of the oracle's OpenMP loops from here on (for timing)."""
    lib().orc_set_threads(int(n))


# ---------------------------------------------------------------- random
def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xffffffff for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xffffffff for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def u53(hi, lo):
    return lib().orc_u53(int(hi), int(lo))


def accept_u(seed, step, a, b):
    return lib().orc_accept_u(int(seed), int(step), int(a), int(b))


# ---------------------------------------------------------------- kernel
def kernel_W(r, h):
    return lib().orc_kernel_W(float(r), float(h))


def lam(d, hi, hj):
    return lib().orc_lambda(float(d), float(hi), float(hj))


# ---------------------------------------------------------------- gravity
def gravity(x, y, z, m, G, eps, query=None, want_norm=False):
    """Self-gravity (a, phi) for all particles or a query subset."""
    x, y, z, m = _f64(x), _f64(y), _f64(z), _f64(m)
    n = x.size
    if query is None:
        nq, qp = n, None
    else:
        query = np.ascontiguousarray(query, dtype=np.int64)
        nq, qp = query.size, query.ctypes.data_as(_i64p)
    ax, ay, az, pot = (np.zeros(nq) for _ in range(4))
    an = np.zeros(nq) if want_norm else None
    lib().orc_gravity(n, _d(x), _d(y), _d(z), _d(m), float(G), float(eps), nq, qp,
                      _d(ax), _d(ay), _d(az), _d(pot), _d(an) if want_norm else None)
    if want_norm:
        return ax, ay, az, pot, an
    return ax, ay, az, pot


def tree_gravity(x, y, z, m, a_old, G, eps, alpha, query=None):
    """Tree self-gravity (a, phi) with the relative opening criterion; a_old =
    (ax, ay, az) of the previous force computation.  query: None (all) or
    particle indices.  Returns ax, ay, az, pot (per query) and the number of
    source terms summed over the groups walked."""
    x, y, z, m = _f64(x), _f64(y), _f64(z), _f64(m)
    ox, oy, oz = (_f64(v) for v in a_old)
    n = x.size
    if query is None:
        nq, qp = n, None
    else:
        query = np.ascontiguousarray(query, dtype=np.int64)
        nq, qp = query.size, query.ctypes.data_as(_i64p)
    ax, ay, az, pot = (np.zeros(nq) for _ in range(4))
    terms = C.c_int64(0)
    lib().orc_tree_gravity(n, _d(x), _d(y), _d(z), _d(m), _d(ox), _d(oy), _d(oz), float(G),
                           float(eps), float(alpha), nq, qp, _d(ax), _d(ay), _d(az), _d(pot),
                           C.byref(terms))
    return ax, ay, az, pot, int(terms.value)


def octree_gravity(x, y, z, m, a_old, G, eps, alpha, query=None):
    """The paper's tree: a geometric oct-tree walked per particle with the
    relative opening criterion.  Returns ax, ay, az, pot (per query) and the
    number of source terms summed."""
    x, y, z, m = _f64(x), _f64(y), _f64(z), _f64(m)
    ox, oy, oz = (_f64(v) for v in a_old)
    n = x.size
    if query is None:
        nq, qp = n, None
    else:
        query = np.ascontiguousarray(query, dtype=np.int64)
        nq, qp = query.size, query.ctypes.data_as(_i64p)
    ax, ay, az, pot = (np.zeros(nq) for _ in range(4))
    terms = C.c_int64(0)
    lib().orc_octree_gravity(n, _d(x), _d(y), _d(z), _d(m), _d(ox), _d(oy), _d(oz), float(G),
                             float(eps), float(alpha), nq, qp, _d(ax), _d(ay), _d(az), _d(pot),
                             C.byref(terms))
    return ax, ay, az, pot, int(terms.value)


def host_nfw(x, y, z, G, rho_s, r_s, c):
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.size
    ax, ay, az, pot = (np.zeros(n) for _ in range(4))
    cc = (C.c_double * 3)(*[float(v) for v in c])
    lib().orc_host_nfw(n, _d(x), _d(y), _d(z), float(G), float(rho_s), float(r_s),
                       cc, _d(ax), _d(ay), _d(az), _d(pot))
    return ax, ay, az, pot


def host_hernquist(x, y, z, G, M, a, c):
    x, y, z = _f64(x), _f64(y), _f64(z)
    out = [np.zeros(x.size) for _ in range(4)]
    cc = (C.c_double * 3)(*[float(v) for v in c])
    lib().orc_host_hernquist(x.size, _d(x), _d(y), _d(z), float(G), float(M), float(a), cc,
                             *[_d(o) for o in out])
    return tuple(out)


def host_disk(x, y, z, G, M, a, b, c):
    x, y, z = _f64(x), _f64(y), _f64(z)
    out = [np.zeros(x.size) for _ in range(4)]
    cc = (C.c_double * 3)(*[float(v) for v in c])
    lib().orc_host_disk(x.size, _d(x), _d(y), _d(z), float(G), float(M), float(a), float(b), cc,
                        *[_d(o) for o in out])
    return tuple(out)


def host_field(x, y, z, p):
    """Total host acceleration and potential of parameter set p."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    out = [np.zeros(x.size) for _ in range(4)]
    lib().orc_host_field(x.size, _d(x), _d(y), _d(z), C.addressof(p), *[_d(o) for o in out])
    return tuple(out)


# ---------------------------------------------------------------- kNN
def knn(x, y, z, ids, k, query=None, want_list=False):
    x, y, z = _f64(x), _f64(y), _f64(z)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    n = x.size
    if query is None:
        nq, qp = n, None
    else:
        query = np.ascontiguousarray(query, dtype=np.int64)
        nq, qp = query.size, query.ctypes.data_as(_i64p)
    h = np.zeros(nq)
    nbr = np.zeros((nq, k), dtype=np.uint32) if want_list else None
    lib().orc_knn(n, _d(x), _d(y), _d(z), ids.ctypes.data_as(_u32p), int(k), nq, qp,
                  _d(h), nbr.ctypes.data_as(_u32p) if want_list else None)
    return (h, nbr) if want_list else h


def knn_grid(x, y, z, ids, k):
    """h of every particle from the grid search (equal to knn's)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    h = np.zeros(x.size)
    lib().orc_knn_grid(x.size, _d(x), _d(y), _d(z), ids.ctypes.data_as(_u32p), int(k), _d(h))
    return h


def knn_tree(x, y, z, ids, k, want_list=False):
    """h (and the neighbour lists) of every particle from the k-d tree search
    (equal to knn's)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    h = np.zeros(x.size)
    nbr = np.zeros((x.size, k), dtype=np.uint32) if want_list else None
    lib().orc_knn_tree(x.size, _d(x), _d(y), _d(z), ids.ctypes.data_as(_u32p), int(k), _d(h),
                       nbr.ctypes.data_as(_u32p) if want_list else None)
    return (h, nbr) if want_list else h


# ---------------------------------------------------------------- scatter
def sigma(sigma_m, sigma_w, g):
    return lib().orc_sigma(float(sigma_m), float(sigma_w), float(g))


def find_events(x, y, z, vx, vy, vz, m, ids, h, sigma_m, dt, seed, step, qmask=None,
                sigma_w=0.0):
    """Events (structured array in (a, b) order), pair count, count of P > 1."""
    arrs = [_f64(a) for a in (x, y, z, vx, vy, vz, m)]
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    h = _f64(h)
    n = arrs[0].size
    qm = None
    if qmask is not None:
        qmask = np.ascontiguousarray(qmask, dtype=np.uint8)
        qm = qmask.ctypes.data_as(_u8p)
    npairs, npgt1 = C.c_int64(0), C.c_int64(0)
    args = [n] + [_d(a) for a in arrs] + [ids.ctypes.data_as(_u32p), _d(h), float(sigma_m),
                                          float(sigma_w), float(dt), int(seed), int(step), qm]
    found = lib().orc_find_events(*args, None, 0, C.byref(npairs), C.byref(npgt1))
    ev = np.zeros(max(found, 1), dtype=EVENT_DTYPE)
    found2 = lib().orc_find_events(*args, ev.ctypes.data, found, None, None)
    assert found2 == found
    return ev[:found], int(npairs.value), int(npgt1.value)


def find_events_sweep(x, y, z, vx, vy, vz, m, ids, h, sigma_m, dt, seed, step, sigma_w=0.0):
    """find_events over all pairs, from the x-sorted sweep (equal results)."""
    arrs = [_f64(a) for a in (x, y, z, vx, vy, vz, m)]
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    h = _f64(h)
    n = arrs[0].size
    npairs, npgt1 = C.c_int64(0), C.c_int64(0)
    args = [n] + [_d(a) for a in arrs] + [ids.ctypes.data_as(_u32p), _d(h), float(sigma_m),
                                          float(sigma_w), float(dt), int(seed), int(step)]
    found = lib().orc_find_events_sweep(*args, None, 0, C.byref(npairs), C.byref(npgt1))
    ev = np.zeros(max(found, 1), dtype=EVENT_DTYPE)
    found2 = lib().orc_find_events_sweep(*args, ev.ctypes.data, found, None, None)
    assert found2 == found
    return ev[:found], int(npairs.value), int(npgt1.value)


def find_events_tree(x, y, z, vx, vy, vz, m, ids, h, sigma_m, dt, seed, step, sigma_w=0.0):
    """find_events over all pairs, from the k-d tree range search (equal results)."""
    arrs = [_f64(a) for a in (x, y, z, vx, vy, vz, m)]
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    h = _f64(h)
    n = arrs[0].size
    npairs, npgt1 = C.c_int64(0), C.c_int64(0)
    args = [n] + [_d(a) for a in arrs] + [ids.ctypes.data_as(_u32p), _d(h), float(sigma_m),
                                          float(sigma_w), float(dt), int(seed), int(step)]
    cap = max(16, n // 64)
    ev = np.zeros(cap, dtype=EVENT_DTYPE)
    found = lib().orc_find_events_tree(*args, ev.ctypes.data, cap, C.byref(npairs),
                                       C.byref(npgt1))
    if found > cap:
        ev = np.zeros(found, dtype=EVENT_DTYPE)
        found2 = lib().orc_find_events_tree(*args, ev.ctypes.data, found, None, None)
        assert found2 == found
    return ev[:found], int(npairs.value), int(npgt1.value)


def central_density(x, y, z, m, phi_self, radius):
    """(centre index, count, mass) within `radius` of the lowest-phi particle."""
    x, y, z, m, phi_self = (_f64(a) for a in (x, y, z, m, phi_self))
    c, cnt, mass = C.c_int64(0), C.c_int64(0), C.c_double(0.0)
    lib().orc_central_density(x.size, _d(x), _d(y), _d(z), _d(m), _d(phi_self), float(radius),
                              C.byref(c), C.byref(cnt), C.byref(mass))
    return int(c.value), int(cnt.value), float(mass.value)


def tidal_radius(x, y, z, m, phi_self, p):
    """(r_tidal, mass within it, centre index, status) in the host of p."""
    x, y, z, m, phi_self = (_f64(a) for a in (x, y, z, m, phi_self))
    r, mass, c = C.c_double(0.0), C.c_double(0.0), C.c_int64(0)
    st = lib().orc_tidal_radius(x.size, _d(x), _d(y), _d(z), _d(m), _d(phi_self), C.addressof(p),
                                C.byref(r), C.byref(mass), C.byref(c))
    return float(r.value), float(mass.value), int(c.value), int(st)


def kick_pair(seed, step, a, b, ma, mb, va, vb):
    va = (C.c_double * 3)(*[float(v) for v in va])
    vb = (C.c_double * 3)(*[float(v) for v in vb])
    lib().orc_kick_pair(int(seed), int(step), int(a), int(b), float(ma), float(mb), va, vb)
    return np.array(list(va)), np.array(list(vb))


def apply_events(ev, m, vx, vy, vz, seed, step):
    """Applies events (in (a, b) order) in place to vx, vy, vz."""
    ev = np.ascontiguousarray(ev, dtype=EVENT_DTYPE)
    for a in (vx, vy, vz):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_apply_events(ev.size, ev.ctypes.data, _d(_f64(m)), _d(vx), _d(vy), _d(vz),
                           int(seed), int(step))


def diag(vx, vy, vz, m, pot, pext=None):
    out = np.zeros(6)
    vx, vy, vz, m, pot = (_f64(a) for a in (vx, vy, vz, m, pot))
    pe = _d(_f64(pext)) if pext is not None else None
    lib().orc_diag(vx.size, _d(vx), _d(vy), _d(vz), _d(m), _d(pot), pe, _d(out))
    return dict(K=out[0], W=out[1], Eext=out[2], px=out[3], py=out[4], pz=out[5])


# ---------------------------------------------------------------- step
def make_params(G=1.0, eps=0.01, sigma_m=1.0, dt=1e-3, k=32, seed=0, host=None, sigma_w=0.0,
                boundary=None, steps=None, tree_alpha=0.0):
    """host: None, an NFW dict (rho_s, r_s, center), or with "hern" = (M, a)
    and "disks" = [(M, a, b), ...] the Milky-Way host.  boundary: None or a
    dict (r, center) for the reflecting sphere.  steps: None (one KDK step of
    dt) or a dict (eta, max_bin, dt_min) for a cycle of block time steps.
    tree_alpha > 0: self-gravity through the tree (a_old = the state's a)."""
    p = OrcParams()
    p.G, p.eps, p.sigma_m, p.dt, p.k, p.seed = G, eps, sigma_m, dt, k, seed
    p.sigma_w = float(sigma_w)
    p.tree_alpha = float(tree_alpha)
    if steps is not None:
        p.eta = float(steps["eta"])
        p.max_bin = int(steps["max_bin"])
        p.dt_min = float(steps.get("dt_min", 0.0))
    if boundary is not None:
        p.boundary_r = float(boundary["r"])
        p.boundary_c = (C.c_double * 3)(*[float(v) for v in boundary.get("center", (0, 0, 0))])
    if host is None:
        p.host_kind = 0
        p.host_rho_s, p.host_r_s = 0.0, 1.0
        p.host_c = (C.c_double * 3)(0.0, 0.0, 0.0)
    else:
        p.host_kind = 2 if ("hern" in host or "disks" in host) else 1
        p.host_rho_s, p.host_r_s = float(host["rho_s"]), float(host["r_s"])
        p.host_c = (C.c_double * 3)(*[float(v) for v in host["center"]])
        if "hern" in host:
            p.host_hern_M, p.host_hern_a = (float(v) for v in host["hern"])
        for d, disk in enumerate(host.get("disks", ())):
            for c in range(3):
                p.host_disk[d][c] = float(disk[c])
    return p


def time_bin(p, ax, ay, az):
    """orc_bin for each particle: the time-step bin from the accelerations."""
    ax, ay, az = (np.asarray(v, dtype=np.float64) for v in (ax, ay, az))
    return np.array([lib().orc_bin(p.dt, p.eta, p.eps, p.dt_min, p.max_bin, a, b, c)
                     for a, b, c in zip(ax, ay, az)], dtype=np.int32)


def total_accel(s, p):
    """a and pot (self + host) at the state's positions, written into s."""
    ax, ay, az, pot = gravity(s["x"], s["y"], s["z"], s["m"], p.G, p.eps)
    if p.host_kind != 0:
        hx, hy, hz, hp = host_field(s["x"], s["y"], s["z"], p)
        ax, ay, az, pot = ax + hx, ay + hy, az + hz, pot + hp
    s["ax"], s["ay"], s["az"], s["pot"] = ax, ay, az, pot
    return s


def kick_drift(s, p):
    """K(dt/2) D(dt) of a fixed step on the dict-of-arrays state s (in place)."""
    for key in ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az"):
        s[key] = np.array(s[key], dtype=np.float64)
    lib().orc_kick_drift(s["x"].size, *[_d(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz",
                                                           "ax", "ay", "az")], C.byref(p))


def close_kick(s, p):
    """The closing K(dt/2) with the state's a (in place)."""
    for key in ("vx", "vy", "vz", "ax", "ay", "az"):
        s[key] = np.array(s[key], dtype=np.float64)
    lib().orc_close_kick(s["x"].size, *[_d(s[k]) for k in ("vx", "vy", "vz", "ax", "ay", "az")],
                         C.byref(p))


def kdk_step(s, p, step, ev_cap=1 << 20):
    """One full step on the dict-of-arrays state s (modified in place)."""
    n = s["x"].size
    for key in ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az", "pot", "m"):
        s[key] = _f64(s[key]).copy() if not s[key].flags.writeable else _f64(s[key])
    s.setdefault("h", np.zeros(n))
    ids = np.ascontiguousarray(s["id"], dtype=np.uint32)
    ev = np.zeros(max(ev_cap, 1), dtype=EVENT_DTYPE)
    found = lib().orc_kdk_step(n, *[_d(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m")],
                               ids.ctypes.data_as(_u32p),
                               *[_d(s[k]) for k in ("ax", "ay", "az", "pot", "h")],
                               C.byref(p), int(step), ev.ctypes.data, ev_cap)
    if found < 0:
        raise RuntimeError("event capacity exceeded in oracle step")
    return ev[:found]
