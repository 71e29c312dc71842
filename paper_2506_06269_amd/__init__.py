"""Python binding of libsidm (the MI355X SIDM N-body step).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libsidm.so.  PyTorch supplies device memory (tensors on a ROCm
device) and the current HIP stream.  The functions carry the C names:

    ctx = sidm_create(device, max_particles, max_halos)
    sidm_gravity(ctx, halos, state, prec)
    sidm_knn_h(ctx, halos, state, nbr=None)
    sidm_scatter(ctx, halos, state, step, events=None, want_count=False)
    sidm_kdk_step(ctx, halos, state, step, prec, diag=None)
    sidm_diagnostics(ctx, halos, state, diag)
    sidm_destroy(ctx)

`halos` is a sequence of dicts with the sidm_halo fields; `state` is a dict of
float64/uint32 device tensors (x, y, z, vx, vy, vz, m, id, ax, ay, az, pot, h).
There is no CPU fallback: if libsidm.so is missing the import fails.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsidm.so")

SIDM_OK = 0
SIDM_ERR_INVALID = -1
SIDM_ERR_NOMEM = -2
SIDM_ERR_HIP = -3
SIDM_ERR_CAPACITY = -4
SIDM_ERR_UNSUPPORTED = -5
SIDM_PREC_FP64 = 0
SIDM_PREC_MIXED = 1
SIDM_MAX_K = 128
SIDM_DEV_EVENT_OVERFLOW = 1
SIDM_DEV_KNN_OVERFLOW = 2
SIDM_DEV_NONFINITE = 4
SIDM_DEV_UNEQUAL_MASS = 8
SIDM_DEV_DUPLICATE_ID = 16
SIDM_DEV_STALE_GRAPH = 32

EXPORTED = ("sidm_create", "sidm_destroy", "sidm_set_event_capacity", "sidm_status_string",
            "sidm_last_error", "sidm_gravity", "sidm_knn_h", "sidm_scatter", "sidm_kdk_step",
            "sidm_diagnostics", "sidm_central_density", "sidm_tidal_radius", "sidm_enable_timing",
            "sidm_pass_times", "sidm_last_events", "sidm_take_status", "sidm_gravity_static",
            "sidm_set_launch_shape", "sidm_autotune", "sidm_set_symmetric")
SIDM_TUNE_FORCE = 1
SIDM_TUNE_QUICK = 2
SIDM_TUNE_CACHE_ONLY = 4
TILES_CACHE = os.path.join(HERE, "tiles.json")   # tuned launch shapes (MI355X entries)
# launch shapes of the gravity tiles: (i-particles per thread, threads per block)
SHAPES = [(i, t) for t in (128, 256, 512) for i in (2, 4, 8)]
SIDM_STATIC_MAX_N = 65536
PASS_NAMES = ("kick_drift", "gravity", "gravity_tiles", "cell_list", "knn", "pairs", "kicks",
              "diag")


class SidmHalo(C.Structure):
    _fields_ = [("offset", C.c_int64), ("n", C.c_int64), ("G", C.c_double),
                ("eps", C.c_double), ("sigma_m", C.c_double), ("dt", C.c_double),
                ("k", C.c_int32), ("host_kind", C.c_int32), ("seed", C.c_uint64),
                ("host_rho_s", C.c_double), ("host_r_s", C.c_double),
                ("host_center", C.c_double * 3), ("sigma_w", C.c_double),
                ("host_hern_M", C.c_double), ("host_hern_a", C.c_double),
                ("host_disk", (C.c_double * 3) * 4), ("boundary_r", C.c_double),
                ("boundary_center", C.c_double * 3), ("eta", C.c_double), ("dt_min", C.c_double),
                ("max_bin", C.c_int32), ("reserved", C.c_int32), ("tree_alpha", C.c_double)]


class SidmState(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in ("x", "y", "z", "vx", "vy", "vz", "m", "id",
                                          "ax", "ay", "az", "pot", "h")]


class SidmDiag(C.Structure):
    _fields_ = [("K", C.c_double), ("W", C.c_double), ("Eext", C.c_double),
                ("px", C.c_double), ("py", C.c_double), ("pz", C.c_double),
                ("n_events", C.c_int64), ("n_rounds", C.c_int64), ("n_pairs", C.c_int64),
                ("n_p_gt1", C.c_int64), ("status", C.c_int32), ("reserved", C.c_int32),
                ("n_grav_terms", C.c_int64), ("n_candidates", C.c_int64)]


class SidmTuneResult(C.Structure):
    _fields_ = [("ireg", C.c_int32), ("threads", C.c_int32), ("persistent", C.c_int32),
                ("from_cache", C.c_int32), ("n_tried", C.c_int32), ("reserved", C.c_int32),
                ("ms", C.c_double), ("ms_default", C.c_double), ("key", C.c_char * 96)]


class SidmCenter(C.Structure):
    _fields_ = [("x", C.c_double), ("y", C.c_double), ("z", C.c_double), ("mass", C.c_double),
                ("index", C.c_int64), ("count", C.c_int64)]


class SidmTidal(C.Structure):
    _fields_ = [("r_tidal", C.c_double), ("mass", C.c_double), ("x", C.c_double),
                ("y", C.c_double), ("z", C.c_double), ("index", C.c_int64),
                ("status", C.c_int32), ("reserved", C.c_int32)]


DIAG_BYTES = C.sizeof(SidmDiag)
CENTER_BYTES = C.sizeof(SidmCenter)
EVENT_BYTES = 16
DIAG_FIELDS = [f for f, _ in SidmDiag._fields_]

_lib = None


class SidmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def lib():
    """Loads libsidm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32
        hp = C.POINTER(SidmHalo)
        sp = C.POINTER(SidmState)
        L.sidm_create.argtypes = [C.POINTER(vp), C.c_int, i64, i32]
        L.sidm_destroy.argtypes = [vp]
        L.sidm_destroy.restype = None
        L.sidm_set_event_capacity.argtypes = [vp, i64]
        L.sidm_status_string.argtypes = [C.c_int]
        L.sidm_status_string.restype = C.c_char_p
        L.sidm_last_error.argtypes = [vp]
        L.sidm_last_error.restype = C.c_char_p
        L.sidm_gravity.argtypes = [vp, hp, i32, sp, C.c_int, vp]
        L.sidm_knn_h.argtypes = [vp, hp, i32, sp, vp, vp]
        L.sidm_scatter.argtypes = [vp, hp, i32, sp, u32, vp, i64, C.POINTER(i64), vp]
        L.sidm_kdk_step.argtypes = [vp, hp, i32, sp, u32, C.c_int, vp, vp]
        L.sidm_diagnostics.argtypes = [vp, hp, i32, sp, vp, vp]
        L.sidm_central_density.argtypes = [vp, hp, i32, sp, C.POINTER(C.c_double), vp, vp]
        L.sidm_tidal_radius.argtypes = [vp, hp, i32, sp, vp, vp]
        L.sidm_enable_timing.argtypes = [vp, C.c_int]
        L.sidm_pass_times.argtypes = [vp, C.POINTER(C.c_double)]
        L.sidm_last_events.argtypes = [vp, vp, i64, C.POINTER(i64), vp]
        L.sidm_take_status.argtypes = [vp, C.POINTER(i32)]
        L.sidm_gravity_static.argtypes = [hp, sp, C.c_int, vp]
        L.sidm_set_launch_shape.argtypes = [vp, i32, i32, i32]
        L.sidm_set_symmetric.argtypes = [vp, i64]
        L.sidm_autotune.argtypes = [vp, hp, i32, sp, C.c_int, C.c_char_p, i32,
                                    C.POINTER(SidmTuneResult), vp]
        for name in EXPORTED:
            if name not in ("sidm_destroy", "sidm_status_string", "sidm_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


class Context:
    def __init__(self, handle, device):
        self.handle = handle
        self.device = device

    def __del__(self):
        try:
            sidm_destroy(self)
        except Exception:
            pass


def _check(ctx, status):
    if status != SIDM_OK:
        L = lib()
        msg = L.sidm_last_error(ctx.handle if ctx else None)
        text = (msg.decode() if msg else "") or L.sidm_status_string(status).decode()
        raise SidmError(status, text)


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(int(stream))


def make_halos(halos):
    arr = (SidmHalo * len(halos))()
    for i, h in enumerate(halos):
        host = h.get("host")
        arr[i].offset = int(h.get("offset", 0))
        arr[i].n = int(h["n"])
        arr[i].G = float(h.get("G", 1.0))
        arr[i].eps = float(h["eps"])
        arr[i].sigma_m = float(h.get("sigma_m", 0.0))
        arr[i].sigma_w = float(h.get("sigma_w", 0.0))
        arr[i].dt = float(h.get("dt", 0.0))
        arr[i].k = int(h.get("k", 0))
        arr[i].seed = int(h.get("seed", 0))
        if host is not None:
            arr[i].host_kind = 2 if ("hern" in host or "disks" in host) else 1
            arr[i].host_rho_s = float(host["rho_s"])
            arr[i].host_r_s = float(host["r_s"])
            for c in range(3):
                arr[i].host_center[c] = float(host["center"][c])
            if "hern" in host:
                arr[i].host_hern_M, arr[i].host_hern_a = (float(v) for v in host["hern"])
            for d, disk in enumerate(host.get("disks", ())):
                for c in range(3):
                    arr[i].host_disk[d][c] = float(disk[c])
        else:
            arr[i].host_kind = int(h.get("host_kind", 0))
        bnd = h.get("boundary")
        if bnd is not None:
            arr[i].boundary_r = float(bnd["r"])
            for c in range(3):
                arr[i].boundary_center[c] = float(bnd.get("center", (0.0, 0.0, 0.0))[c])
        arr[i].tree_alpha = float(h.get("tree_alpha", 0.0))
        steps = h.get("steps")
        if steps is not None:
            arr[i].eta = float(steps["eta"])
            arr[i].max_bin = int(steps["max_bin"])
            arr[i].dt_min = float(steps.get("dt_min", 0.0))
    return arr


def make_state(state):
    s = SidmState()
    for f, _ in SidmState._fields_:
        t = state.get(f)
        setattr(s, f, None if t is None else t.data_ptr())
    return s


def sidm_create(device=0, max_particles=1 << 20, max_halos=1):
    h = C.c_void_p()
    st = lib().sidm_create(C.byref(h), int(device), int(max_particles), int(max_halos))
    if st != SIDM_OK:
        raise SidmError(st, f"sidm_create failed: {lib().sidm_status_string(st).decode()}")
    return Context(h, device)


def sidm_destroy(ctx):
    if ctx is not None and ctx.handle:
        lib().sidm_destroy(ctx.handle)
        ctx.handle = None


def sidm_status_string(status):
    return lib().sidm_status_string(int(status)).decode()


def sidm_last_error(ctx):
    msg = lib().sidm_last_error(ctx.handle if ctx is not None else None)
    return msg.decode() if msg else ""


def sidm_set_event_capacity(ctx, max_events):
    _check(ctx, lib().sidm_set_event_capacity(ctx.handle, int(max_events)))


def sidm_gravity(ctx, halos, state, prec=SIDM_PREC_MIXED, stream=None):
    H = make_halos(halos)
    S = make_state(state)
    _check(ctx, lib().sidm_gravity(ctx.handle, H, len(halos), C.byref(S), int(prec),
                                   _stream(stream)))


def sidm_gravity_static(halo, state, prec=SIDM_PREC_MIXED, stream=None):
    """The gravity pass for one halo (n <= SIDM_STATIC_MAX_N) without a context
    and without any allocation (the library's fixed scratch array)."""
    H = make_halos([halo])
    S = make_state(state)
    _check(None, lib().sidm_gravity_static(H, C.byref(S), int(prec), _stream(stream)))


def sidm_set_launch_shape(ctx, ireg, threads, persistent=False):
    """Launch shape of the direct-sum gravity tiles (see SHAPES)."""
    _check(ctx, lib().sidm_set_launch_shape(ctx.handle, int(ireg), int(threads),
                                            1 if persistent else 0))


def sidm_set_symmetric(ctx, min_n):
    """Mixed-precision direct sums of halos with at least min_n particles use
    the symmetric tiles (0: never)."""
    _check(ctx, lib().sidm_set_symmetric(ctx.handle, int(min_n)))


def sidm_autotune(ctx, halos, state, prec=SIDM_PREC_MIXED, cache_path=None, flags=0,
                  stream=None):
    """Chooses the launch shape for these halos (from the cache or by timing
    every shape), leaves it on the context and computes the gravity with it.
    Returns the result as a dict."""
    H = make_halos(halos)
    S = make_state(state)
    res = SidmTuneResult()
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(ctx, lib().sidm_autotune(ctx.handle, H, len(halos), C.byref(S), int(prec), path,
                                    int(flags), C.byref(res), _stream(stream)))
    out = {f: getattr(res, f) for f, _ in SidmTuneResult._fields_ if f != "reserved"}
    out["key"] = res.key.decode()
    return out


def sidm_knn_h(ctx, halos, state, nbr=None, stream=None):
    H = make_halos(halos)
    S = make_state(state)
    _check(ctx, lib().sidm_knn_h(ctx.handle, H, len(halos), C.byref(S),
                                 None if nbr is None else C.c_void_p(nbr.data_ptr()),
                                 _stream(stream)))


def sidm_scatter(ctx, halos, state, step, events=None, want_count=False, stream=None):
    """events: optional uint8 device tensor of cap*16 bytes (sidm_event records).
    Returns the number of events if want_count (this waits for the device)."""
    H = make_halos(halos)
    S = make_state(state)
    cnt = C.c_int64(0)
    cap = 0 if events is None else events.numel() * events.element_size() // EVENT_BYTES
    _check(ctx, lib().sidm_scatter(ctx.handle, H, len(halos), C.byref(S), int(step),
                                   None if events is None else C.c_void_p(events.data_ptr()),
                                   int(cap), C.byref(cnt) if want_count else None,
                                   _stream(stream)))
    return int(cnt.value) if want_count else None


def sidm_last_events(ctx, events, want_count=False, stream=None):
    """Copies the events of the last scattering pass on the context into
    `events` (uint8 device tensor of cap*16 bytes).  Returns the number of
    events if want_count (this waits for the device)."""
    cnt = C.c_int64(0)
    cap = events.numel() * events.element_size() // EVENT_BYTES
    _check(ctx, lib().sidm_last_events(ctx.handle, C.c_void_p(events.data_ptr()), int(cap),
                                       C.byref(cnt) if want_count else None, _stream(stream)))
    return int(cnt.value) if want_count else None


def sidm_take_status(ctx):
    """Waits for the device; the SIDM_DEV_* bits not yet reported (cleared)."""
    bits = C.c_int32(0)
    _check(ctx, lib().sidm_take_status(ctx.handle, C.byref(bits)))
    return int(bits.value)


def sidm_kdk_step(ctx, halos, state, step, prec=SIDM_PREC_MIXED, diag=None, stream=None):
    H = make_halos(halos)
    S = make_state(state)
    _check(ctx, lib().sidm_kdk_step(ctx.handle, H, len(halos), C.byref(S), int(step), int(prec),
                                    None if diag is None else C.c_void_p(diag.data_ptr()),
                                    _stream(stream)))


def sidm_diagnostics(ctx, halos, state, diag, stream=None):
    H = make_halos(halos)
    S = make_state(state)
    _check(ctx, lib().sidm_diagnostics(ctx.handle, H, len(halos), C.byref(S),
                                       C.c_void_p(diag.data_ptr()), _stream(stream)))


def sidm_central_density(ctx, halos, state, radius, out=None, stream=None):
    """Centre (lowest self-potential) and the number and mass within `radius`
    (one value or one per halo) of it, per halo.  Returns a list of dicts
    (synchronises) unless a device buffer `out` is given."""
    H = make_halos(halos)
    S = make_state(state)
    r = list(radius) if hasattr(radius, "__len__") else [float(radius)] * len(halos)
    rad = (C.c_double * len(halos))(*[float(v) for v in r])
    buf = out if out is not None else center_buffer(len(halos))
    _check(ctx, lib().sidm_central_density(ctx.handle, H, len(halos), C.byref(S), rad,
                                           C.c_void_p(buf.data_ptr()), _stream(stream)))
    if out is not None:
        return None
    raw = bytes(buf.cpu().numpy().tobytes())
    res = []
    for i in range(len(halos)):
        c = SidmCenter.from_buffer_copy(raw[i * CENTER_BYTES:(i + 1) * CENTER_BYTES])
        res.append({f: getattr(c, f) for f, _ in SidmCenter._fields_})
    return res


def sidm_tidal_radius(ctx, halos, state, stream=None):
    """Tidal radius of each halo in its host (synchronises); list of dicts."""
    import torch
    H = make_halos(halos)
    S = make_state(state)
    nb = C.sizeof(SidmTidal)
    buf = torch.zeros(len(halos) * nb, dtype=torch.uint8, device="cuda")
    _check(ctx, lib().sidm_tidal_radius(ctx.handle, H, len(halos), C.byref(S),
                                        C.c_void_p(buf.data_ptr()), _stream(stream)))
    raw = bytes(buf.cpu().numpy().tobytes())
    out = []
    for i in range(len(halos)):
        t = SidmTidal.from_buffer_copy(raw[i * nb:(i + 1) * nb])
        out.append({f: getattr(t, f) for f, _ in SidmTidal._fields_})
    return out


def center_buffer(n_halos, device="cuda"):
    import torch
    return torch.zeros(n_halos * CENTER_BYTES, dtype=torch.uint8, device=device)


def sidm_enable_timing(ctx, on=True):
    _check(ctx, lib().sidm_enable_timing(ctx.handle, 1 if on else 0))


def sidm_pass_times(ctx):
    """Per-pass milliseconds of the last timed step (waits for it)."""
    out = (C.c_double * len(PASS_NAMES))()
    _check(ctx, lib().sidm_pass_times(ctx.handle, out))
    return dict(zip(PASS_NAMES, list(out)))


# ------------------------------------------------------------------ helpers
def diag_buffer(n_halos, device="cuda"):
    import torch
    return torch.zeros(n_halos * DIAG_BYTES, dtype=torch.uint8, device=device)


def read_diag(buf):
    """Decodes a diag buffer (device or host uint8 tensor) into dicts."""
    raw = bytes(buf.cpu().numpy().tobytes())
    out = []
    for i in range(len(raw) // DIAG_BYTES):
        d = SidmDiag.from_buffer_copy(raw[i * DIAG_BYTES:(i + 1) * DIAG_BYTES])
        out.append({f: getattr(d, f) for f in DIAG_FIELDS})
    return out


def event_buffer(cap, device="cuda"):
    import torch
    return torch.zeros(cap * EVENT_BYTES, dtype=torch.uint8, device=device)


def read_events(buf, count):
    """Decodes `count` sidm_event records into a numpy structured array."""
    import numpy as np
    dt = np.dtype([("a", np.uint32), ("b", np.uint32), ("halo", np.int32), ("round", np.uint32)])
    raw = buf[:count * EVENT_BYTES].cpu().numpy()
    return raw.view(dt).copy()


def state_to_device(s, device="cuda"):
    """Host dict of numpy arrays -> dict of device tensors with all fields."""
    import numpy as np
    import torch
    n = s["x"].size
    out = {}
    for f in ("x", "y", "z", "vx", "vy", "vz", "m"):
        out[f] = torch.from_numpy(np.ascontiguousarray(s[f], dtype=np.float64)).to(device)
    out["id"] = torch.from_numpy(np.ascontiguousarray(s["id"], dtype=np.uint32).view(np.int32)).to(device)
    for f in ("ax", "ay", "az", "pot", "h"):
        if f in s:
            out[f] = torch.from_numpy(np.ascontiguousarray(s[f], dtype=np.float64)).to(device)
        else:
            out[f] = torch.zeros(n, dtype=torch.float64, device=device)
    return out


def state_to_host(st):
    import numpy as np
    out = {}
    for f, t in st.items():
        a = t.detach().cpu().numpy()
        out[f] = a.view(np.uint32) if f == "id" else a
    return out
