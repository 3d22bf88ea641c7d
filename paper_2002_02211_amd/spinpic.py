"""ctypes binding of libspinpic (include/spinpic.h).

The functions ``pic_init``, ``pic_step``, ``pic_polarization``, ``pic_fields``,
``pic_particles``, ``pic_energy``, ``pic_stats``, ``pic_timing``,
``pic_timing_read`` and ``pic_free`` mirror the C calls one to one: they only
marshal arguments (numpy arrays in, numpy arrays out) and raise ``PicError``
on a negative status.  Every step of the computation runs in the HIP kernels
of the library; there is no fallback path.  Device memory comes from torch's
caching allocator and work is enqueued on torch's current stream.
"""

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspinpic.so")

PIC_OK, PIC_EINVAL, PIC_ECFL, PIC_EHIP, PIC_ECAPACITY, PIC_ENONFINITE, PIC_ESTATE, PIC_ENOMEM = \
    0, -1, -2, -3, -4, -5, -6, -7
PIC_FP64, PIC_FP32_MIXED = 0, 1
PIC_ACC_DEFAULT, PIC_ACC_FP32, PIC_ACC_FP64 = 0, 1, 2
PIC_FLAG_TEST_PARTICLE = 1
PIC_FLAG_DETERMINISTIC = 2
PIC_FLAG_CELL_ROWS = 4
MAX_SPECIES = 4
PIC_MAX_SPECTRUM_BINS = 1024
FIELD_NAMES = ("Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz", "rho")
EXPORTED = ("pic_init", "pic_step", "pic_polarization", "pic_polarization_record",
            "pic_polarization_history", "pic_fields", "pic_particles",
            "pic_spectrum", "pic_spectrum_noalloc", "pic_phase_space", "pic_density", "pic_energy", "pic_stats",
            "pic_particles_cells", "pic_test_poison",
            "pic_window", "pic_timing", "pic_timing_read", "pic_last_error", "pic_free",
            "pic_batch_init", "pic_batch_step", "pic_batch_polarization", "pic_batch_fields",
            "pic_batch_particles", "pic_batch_info", "pic_batch_tuning", "pic_batch_stats",
            "pic_batch_timing", "pic_batch_timing_read", "pic_batch_last_error", "pic_batch_free",
            "pic_track_create", "pic_track_forward", "pic_track_backward", "pic_track_timing",
            "pic_track_last_error", "pic_track_free")

_ERR_NAMES = {PIC_EINVAL: "PIC_EINVAL", PIC_ECFL: "PIC_ECFL", PIC_EHIP: "PIC_EHIP",
              PIC_ECAPACITY: "PIC_ECAPACITY", PIC_ENONFINITE: "PIC_ENONFINITE",
              PIC_ESTATE: "PIC_ESTATE", PIC_ENOMEM: "PIC_ENOMEM"}


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_ERR_NAMES.get(code, "?"), code, msg))
        self.code = code
        self.msg = msg


class Species(ctypes.Structure):
    _fields_ = [("Z", ctypes.c_double), ("mu", ctypes.c_double), ("a", ctypes.c_double)]


class Config(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("d", ctypes.c_double * 3),
        ("dt", ctypes.c_double), ("precision", ctypes.c_int32), ("nspecies", ctypes.c_int32),
        ("sp", Species * MAX_SPECIES), ("tile", ctypes.c_int32 * 3), ("slack", ctypes.c_double),
        ("flags", ctypes.c_int32), ("deposit_acc", ctypes.c_int32),
    ]


class State(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64 * MAX_SPECIES),
                ("particles", ctypes.c_void_p * MAX_SPECIES),
                ("fields", ctypes.c_void_p)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class TrackConfig(ctypes.Structure):
    _fields_ = [("Z", ctypes.c_double), ("mu", ctypes.c_double), ("a", ctypes.c_double),
                ("dt", ctypes.c_double), ("nsteps", ctypes.c_int32), ("checkpoint", ctypes.c_int32),
                ("precision", ctypes.c_int32)]


class WindowConfig(ctypes.Structure):
    _fields_ = [("speed", ctypes.c_double), ("shift_cells", ctypes.c_int32), ("ppc", ctypes.c_int32),
                ("n0", ctypes.c_double), ("ramp_start", ctypes.c_double), ("ramp_len", ctypes.c_double),
                ("s0", ctypes.c_double * 3)]


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


_lib = None


def load_library(path=LIB_PATH):
    """Load libspinpic.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libspinpic.so is not built (%s); run "
                           "`python -m paper_2002_02211_amd.build`" % path)
    # torch ships its own HIP runtime under the same soname; importing it first
    # makes the library bind to that one, so the streams and device pointers
    # torch hands over belong to the runtime the library calls
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.pic_init.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(State),
                             ctypes.POINTER(Allocator), P, ctypes.POINTER(P)]
    lib.pic_step.argtypes = [P, ctypes.c_int32]
    lib.pic_polarization.argtypes = [P, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.pic_polarization_record.argtypes = [P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32]
    lib.pic_polarization_history.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                             ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.pic_fields.argtypes = [P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t]
    lib.pic_particles.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                  ctypes.c_size_t, ctypes.POINTER(ctypes.c_int64)]
    D = ctypes.POINTER(ctypes.c_double)
    lib.pic_spectrum.argtypes = [P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                 D, D, D]
    lib.pic_particles_cells.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                        ctypes.c_size_t, ctypes.POINTER(ctypes.c_int64)]
    lib.pic_test_poison.argtypes = [P, ctypes.c_int32]
    lib.pic_spectrum_noalloc.argtypes = [P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                         D, D, D]
    lib.pic_phase_space.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int32, D]
    lib.pic_density.argtypes = [P, ctypes.c_int32, D, ctypes.c_size_t]
    lib.pic_energy.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.c_int32]
    lib.pic_stats.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]
    lib.pic_window.argtypes = [P, ctypes.POINTER(WindowConfig)]
    lib.pic_timing.argtypes = [P, ctypes.c_int32]
    lib.pic_timing_read.argtypes = [P, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]
    I64 = ctypes.POINTER(ctypes.c_int64)
    I32 = ctypes.POINTER(ctypes.c_int32)
    lib.pic_batch_init.argtypes = [ctypes.c_int32, ctypes.POINTER(Config), ctypes.POINTER(State), ctypes.c_int32,
                                   ctypes.POINTER(Allocator), P, ctypes.POINTER(P)]
    lib.pic_batch_step.argtypes = [P, ctypes.c_int32]
    lib.pic_batch_polarization.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double, D, I64]
    lib.pic_batch_fields.argtypes = [P, ctypes.c_int32, ctypes.c_uint32, D, ctypes.c_size_t]
    lib.pic_batch_particles.argtypes = [P, ctypes.c_int32, ctypes.c_int32, D, ctypes.c_size_t, I64]
    lib.pic_batch_info.argtypes = [P, ctypes.c_int32, I64]
    lib.pic_batch_tuning.argtypes = [P, I32, D, D, ctypes.c_int32, I32]
    lib.pic_batch_stats.argtypes = [P, I64, ctypes.c_int32]
    lib.pic_batch_timing.argtypes = [P, ctypes.c_int32]
    lib.pic_batch_timing_read.argtypes = [P, D, I64, ctypes.c_int32]
    lib.pic_batch_last_error.argtypes = [P]
    lib.pic_batch_last_error.restype = ctypes.c_char_p
    lib.pic_batch_free.argtypes = [P]
    lib.pic_batch_free.restype = None
    lib.pic_track_create.argtypes = [ctypes.POINTER(TrackConfig), ctypes.c_int64,
                                     ctypes.POINTER(Allocator), P, ctypes.POINTER(P)]
    lib.pic_track_forward.argtypes = [P, ctypes.c_double, ctypes.c_double, D, D, D, D, D, D, D]
    lib.pic_track_backward.argtypes = [P, D, D, D, D, D, D]
    lib.pic_track_timing.argtypes = [P, D]
    lib.pic_track_last_error.argtypes = [P]
    lib.pic_track_last_error.restype = ctypes.c_char_p
    lib.pic_track_free.argtypes = [P]
    lib.pic_track_free.restype = None
    lib.pic_last_error.argtypes = [P]
    lib.pic_last_error.restype = ctypes.c_char_p
    lib.pic_free.argtypes = [P]
    lib.pic_free.restype = None
    for name in EXPORTED:
        if name not in ("pic_last_error", "pic_free", "pic_track_last_error", "pic_track_free",
                        "pic_batch_last_error", "pic_batch_free"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(code, ctx=None):
    if code != PIC_OK:
        lib = load_library()
        msg = lib.pic_last_error(ctx)
        raise PicError(code, msg.decode() if msg else "")


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---------------------------------------------------------------- config

def make_config(ndim, n, d, dt, species, precision=PIC_FP64, tile=(0, 0, 0), slack=0.0,
                flags=0, deposit_acc=PIC_ACC_DEFAULT):
    cfg = Config()
    cfg.ndim = int(ndim)
    for a in range(3):
        cfg.n[a] = int(n[a]) if a < len(n) else 1
        cfg.d[a] = float(d[a]) if a < len(d) else 1.0
        cfg.tile[a] = int(tile[a]) if a < len(tile) else 0
    cfg.dt = float(dt)
    cfg.precision = int(precision)
    cfg.nspecies = len(species)
    for s, sp in enumerate(species[:MAX_SPECIES]):
        cfg.sp[s].Z = float(sp["Z"])
        cfg.sp[s].mu = float(sp["mu"])
        cfg.sp[s].a = float(sp["a"])
    cfg.slack = float(slack)
    cfg.flags = int(flags)
    cfg.deposit_acc = int(deposit_acc)
    return cfg


def config_from_spec(spec, precision=None, tile=None, test_particle=False, slack=0.0,
                     deposit_acc=PIC_ACC_DEFAULT, deterministic=False, cell_rows=False):
    """Config from a workload recipe dict (ndim, n, d, dt, species, ...)."""
    if precision is None:
        precision = spec.get("precision", "fp64")
    if isinstance(precision, str):
        precision = {"fp64": PIC_FP64, "fp32": PIC_FP32_MIXED}[precision]
    if tile is None:
        tile = spec.get("tile", (0, 0, 0))
        if spec["ndim"] == 3 and precision == PIC_FP64:
            tile = (0, 0, 0)
    return make_config(spec["ndim"], spec["n"], spec["d"], spec["dt"], spec["species"],
                       precision=precision, tile=tile, slack=slack,
                       flags=((PIC_FLAG_TEST_PARTICLE if test_particle else 0) |
                              (PIC_FLAG_DETERMINISTIC if deterministic else 0) |
                              (PIC_FLAG_CELL_ROWS if cell_rows else 0)),
                       deposit_acc=deposit_acc)


# ---------------------------------------------------------------- torch glue

class _TorchMemory:
    """Device allocator and stream backed by torch's caching allocator."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)

        def _alloc(user, size):
            try:
                return torch.cuda.caching_allocator_alloc(int(size), self.device, self.stream)
            except Exception:   # noqa: BLE001 - reported to C as NULL
                return None

        def _free(user, ptr):
            torch.cuda.caching_allocator_delete(ptr)

        self._alloc_fn = ALLOC_FN(_alloc)
        self._free_fn = FREE_FN(_free)
        self.allocator = Allocator(self._alloc_fn, self._free_fn, None)

    @property
    def stream_handle(self):
        return ctypes.c_void_p(self.stream.cuda_stream)


# ---------------------------------------------------------------- C calls

def _make_state(particles, fields, keep):
    """A State pointing at float64 copies of the arrays (kept alive in keep)."""
    st = State()
    for s in range(MAX_SPECIES):
        if s < len(particles) and particles[s] is not None and len(particles[s]):
            arr = np.ascontiguousarray(particles[s], dtype=np.float64)
            if arr.ndim != 2 or arr.shape[1] not in (10, 13):
                raise ValueError("particles[%d] must have shape (N, 10), or (N, 13) in cell form" % s)
            keep.append(arr)
            st.count[s] = arr.shape[0]
            st.particles[s] = arr.ctypes.data
        else:
            st.count[s] = 0
            st.particles[s] = None
    if fields is not None:
        F = np.ascontiguousarray(fields, dtype=np.float64)
        keep.append(F)
        st.fields = F.ctypes.data
    return st


def pic_init(cfg, particles, fields=None, device=0, memory=None):
    """Create a context.  particles: list of (N, 10) float64 arrays per species
    (x y z ux uy uz sx sy sz w), or with PIC_FLAG_CELL_ROWS (N, 13) arrays
    (cx cy cz ox oy oz ux uy uz sx sy sz w); fields: (6, nz, ny, nx) float64
    or None.
    Returns (ctx, memory) - keep ``memory`` alive as long as the context."""
    lib = load_library()
    keep = []
    st = _make_state(particles, fields, keep)
    if memory is None:
        memory = _TorchMemory(device)
    ctx = ctypes.c_void_p()
    code = lib.pic_init(ctypes.byref(cfg), ctypes.byref(st), ctypes.byref(memory.allocator),
                        memory.stream_handle, ctypes.byref(ctx))
    _check(code, None)
    return ctx, memory


def pic_step(ctx, nsteps=1):
    _check(load_library().pic_step(ctx, int(nsteps)), ctx)


def pic_polarization(ctx, species=-1, ekin_min_mev=-math.inf, ekin_max_mev=math.inf):
    P = np.zeros(3)
    N = ctypes.c_int64()
    _check(load_library().pic_polarization(ctx, int(species), float(ekin_min_mev),
                                           float(ekin_max_mev), _dptr(P), ctypes.byref(N)), ctx)
    return P, int(N.value)


PIC_MAX_RECORD_STEPS = 65536


def pic_polarization_record(ctx, species=-1, ekin_min_mev=-math.inf, ekin_max_mev=math.inf, capacity=1024):
    _check(load_library().pic_polarization_record(ctx, int(species), float(ekin_min_mev), float(ekin_max_mev),
                                                  int(capacity)), ctx)


def pic_polarization_history(ctx, cap):
    """(P, N): the recorded steps' mean spins, shape (n, 3), and counts, shape (n,)."""
    P = np.zeros((max(int(cap), 1), 3))
    N = np.zeros(max(int(cap), 1), dtype=np.int64)
    n = ctypes.c_int32()
    _check(load_library().pic_polarization_history(ctx, _dptr(P), N.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                                   int(cap), ctypes.byref(n)), ctx)
    return P[:n.value].copy(), N[:n.value].copy()


def pic_fields(ctx, mask, cells):
    ncomp = bin(int(mask)).count("1")
    out = np.empty(ncomp * cells)
    _check(load_library().pic_fields(ctx, int(mask), _dptr(out), out.size), ctx)
    return out


def pic_particles(ctx, species, count):
    out = np.empty((count, 11))
    n = ctypes.c_int64()
    _check(load_library().pic_particles(ctx, int(species), _dptr(out), out.size, ctypes.byref(n)), ctx)
    return out[: n.value]


def pic_particles_cells(ctx, species, count):
    """Rows (id, cx cy cz, ox oy oz, u, s, w) sorted by id, every value exact."""
    out = np.empty((count, 14))
    n = ctypes.c_int64()
    _check(load_library().pic_particles_cells(ctx, int(species), _dptr(out), out.size, ctypes.byref(n)), ctx)
    return out[: n.value]


def pic_test_poison(ctx, species):
    _check(load_library().pic_test_poison(ctx, int(species)), ctx)


def pic_spectrum(ctx, species, emin, emax, nbins):
    """(count, weight, spin) per kinetic-energy bin; spin has shape (nbins, 3)."""
    count = np.zeros(int(nbins))
    weight = np.zeros(int(nbins))
    spin = np.zeros((int(nbins), 3))
    _check(load_library().pic_spectrum(ctx, int(species), float(emin), float(emax), int(nbins),
                                       _dptr(count), _dptr(weight), _dptr(spin)), ctx)
    return count, weight, spin


def pic_spectrum_noalloc(ctx, species, emin, emax, nbins):
    """pic_spectrum summed in the library's static device buffer (no allocation)."""
    count = np.zeros(int(nbins))
    weight = np.zeros(int(nbins))
    spin = np.zeros((int(nbins), 3))
    _check(load_library().pic_spectrum_noalloc(ctx, int(species), float(emin), float(emax), int(nbins),
                                               _dptr(count), _dptr(weight), _dptr(spin)), ctx)
    return count, weight, spin


def pic_phase_space(ctx, species, axis, xmin, xmax, nx, comp, pmin, pmax, np_):
    out = np.zeros((int(nx), int(np_)))
    _check(load_library().pic_phase_space(ctx, int(species), int(axis), float(xmin), float(xmax),
                                          int(nx), int(comp), float(pmin), float(pmax), int(np_),
                                          _dptr(out)), ctx)
    return out


def pic_density(ctx, species, cells):
    out = np.empty(int(cells))
    _check(load_library().pic_density(ctx, int(species), _dptr(out), out.size), ctx)
    return out


def pic_energy(ctx, nspecies):
    out = np.empty(nspecies + 2)
    _check(load_library().pic_energy(ctx, _dptr(out), out.size), ctx)
    return out


def pic_stats(ctx):
    out = (ctypes.c_int64 * 13)()
    _check(load_library().pic_stats(ctx, out, 13), ctx)
    return {"steps": out[0], "moved": out[1], "overflow": out[2], "repacks": out[3],
            "particles": out[4], "tile": (out[5], out[6], out[7]),
            "per_species": [out[8], out[9], out[10], out[11]], "shifts": out[12]}


def window_config(speed=1.0, shift_cells=16, ppc=0, n0=0.0, ramp_start=0.0, ramp_len=0.0, s0=(0.0, 1.0, 0.0)):
    w = WindowConfig()
    w.speed = float(speed)
    w.shift_cells = int(shift_cells)
    w.ppc = int(ppc)
    w.n0 = float(n0)
    w.ramp_start = float(ramp_start)
    w.ramp_len = float(ramp_len)
    for i in range(3):
        w.s0[i] = float(s0[i])
    return w


def pic_window(ctx, w):
    _check(load_library().pic_window(ctx, ctypes.byref(w)), ctx)


def _timing_mode(enable, push_only):
    return 0 if not enable else (2 if push_only else 1)


def pic_timing(ctx, enable, push_only=False):
    """Start (every kernel class, or the push only) or stop event timing."""
    _check(load_library().pic_timing(ctx, _timing_mode(enable, push_only)), ctx)


TIMER_NAMES = ("push_deposit", "overflow_push", "insert", "fdtd")


def pic_timing_read(ctx):
    ms = np.zeros(len(TIMER_NAMES))
    n = (ctypes.c_int64 * len(TIMER_NAMES))()
    _check(load_library().pic_timing_read(ctx, _dptr(ms), n, len(TIMER_NAMES)), ctx)
    return {name: (float(ms[i]), int(n[i])) for i, name in enumerate(TIMER_NAMES)}


def pic_free(ctx):
    load_library().pic_free(ctx)


# ---------------------------------------------------------------- convenience

class Simulation:
    """A context plus its shapes: the calls above as methods."""

    def __init__(self, cfg, particles, fields=None, device=0):
        self.cfg = cfg
        self.nspecies = cfg.nspecies
        self.shape = (cfg.n[2] if cfg.ndim == 3 else 1, cfg.n[1], cfg.n[0])
        self.cells = int(np.prod(self.shape))
        self.counts = [len(p) if p is not None else 0 for p in particles]
        self.ctx, self._mem = pic_init(cfg, particles, fields, device=device)

    def step(self, n=1):
        pic_step(self.ctx, n)

    def polarization(self, species=-1, emin=-math.inf, emax=math.inf):
        return pic_polarization(self.ctx, species, emin, emax)

    def record_polarization(self, species=-1, emin=-math.inf, emax=math.inf, capacity=1024):
        """Start a per-step Eq. 4 record of `capacity` steps (0: stop)."""
        pic_polarization_record(self.ctx, species, emin, emax, capacity)
        self._rec_cap = int(capacity)

    def polarization_history(self):
        """The recorded steps since the last call: P (n, 3) and N (n,)."""
        return pic_polarization_history(self.ctx, getattr(self, "_rec_cap", 0))

    def fields(self, names=FIELD_NAMES):
        mask = 0
        for nm in names:
            mask |= 1 << FIELD_NAMES.index(nm)
        out = pic_fields(self.ctx, mask, self.cells)
        order = [nm for nm in FIELD_NAMES if nm in names]
        arr = out.reshape((len(order),) + self.shape)
        return {nm: arr[i] for i, nm in enumerate(order)}

    def particles(self, species):
        """Rows (id, x y z, u, s, w) of the particles in the box, sorted by id."""
        count = self.stats()["per_species"][species]
        return pic_particles(self.ctx, species, count)

    def particles_cells(self, species):
        """Rows (id, cx cy cz, ox oy oz, u, s, w), sorted by id, exact."""
        count = self.stats()["per_species"][species]
        return pic_particles_cells(self.ctx, species, count)

    def poison(self, species):
        pic_test_poison(self.ctx, species)

    def window(self, **kw):
        """Open the x faces and start a moving window (see window_config)."""
        pic_window(self.ctx, window_config(**kw))

    def energy(self):
        return pic_energy(self.ctx, self.nspecies)

    def spectrum(self, species, emin, emax, nbins):
        return pic_spectrum(self.ctx, species, emin, emax, nbins)

    def spectrum_noalloc(self, species, emin, emax, nbins):
        return pic_spectrum_noalloc(self.ctx, species, emin, emax, nbins)

    def phase_space(self, species, axis, xmin, xmax, nx, comp, pmin, pmax, np_):
        return pic_phase_space(self.ctx, species, axis, xmin, xmax, nx, comp, pmin, pmax, np_)

    def density(self, species):
        return pic_density(self.ctx, species, self.cells).reshape(self.shape)

    def stats(self):
        return pic_stats(self.ctx)

    def timing(self, enable=True, push_only=False):
        pic_timing(self.ctx, enable, push_only)

    def timing_read(self):
        return pic_timing_read(self.ctx)

    def close(self):
        if self.ctx is not None:
            pic_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # noqa: BLE001
            pass


# ---------------------------------------------------------------- tracking

def _track_check(code, tr):
    if code != PIC_OK:
        msg = load_library().pic_track_last_error(tr)
        raise PicError(code, msg.decode() if msg else "")


def _rows3(a, n, name):
    arr = np.ascontiguousarray(a, dtype=np.float64)
    if arr.shape != (n, 3):
        raise ValueError("%s must have shape (%d, 3)" % (name, n))
    return arr


class Tracker:
    """Spin tracking of n test particles through the analytic wakefield, and
    the gradient of the final polarization (pic_track_*)."""

    def __init__(self, n, Z=1.0, mu=1836.15267343, a=1.793, dt=0.5, nsteps=4000, checkpoint=100,
                 precision="fp32", device=0):
        lib = load_library()
        self.n = int(n)
        cfg = TrackConfig(float(Z), float(mu), float(a), float(dt), int(nsteps), int(checkpoint),
                          {"fp64": PIC_FP64, "fp32": PIC_FP32_MIXED}[precision])
        self._mem = _TorchMemory(device)
        h = ctypes.c_void_p()
        _track_check(lib.pic_track_create(ctypes.byref(cfg), self.n, ctypes.byref(self._mem.allocator),
                                          self._mem.stream_handle, ctypes.byref(h)), None)
        self.h = h
        self.generation = 0

    def forward(self, E0, kp, x0, u0, s0, want_state=False):
        """Final polarization P (3,), and the final x, u, s if asked."""
        n = self.n
        x0, u0, s0 = _rows3(x0, n, "x0"), _rows3(u0, n, "u0"), _rows3(s0, n, "s0")
        P = np.zeros(3)
        outs = [np.empty((n, 3)) for _ in range(3)] if want_state else [None, None, None]
        ptr = [_dptr(o) if o is not None else None for o in outs]
        _track_check(load_library().pic_track_forward(self.h, float(E0), float(kp), _dptr(x0), _dptr(u0),
                                                      _dptr(s0), _dptr(P), *ptr), self.h)
        self.generation += 1
        return (P, *outs) if want_state else P

    def backward(self, c, per_particle_theta=False):
        """(dJ/dE0, dJ/dkp), dJ/dx0, dJ/du0, dJ/ds0 for J = c . P of the last forward
        run; with per_particle_theta also each particle's (dJ/dE0, dJ/dkp) share."""
        n = self.n
        c = np.ascontiguousarray(c, dtype=np.float64).reshape(3)
        gth = np.zeros(2)
        gx, gu, gs = np.empty((n, 3)), np.empty((n, 3)), np.empty((n, 3))
        each = np.empty((n, 2)) if per_particle_theta else None
        _track_check(load_library().pic_track_backward(self.h, _dptr(c), _dptr(gth), _dptr(gx), _dptr(gu),
                                                       _dptr(gs), _dptr(each) if each is not None else None),
                     self.h)
        out = (gth, gx, gu, gs)
        return out + (each,) if per_particle_theta else out

    def timing(self):
        ms = np.zeros(2)
        _track_check(load_library().pic_track_timing(self.h, _dptr(ms)), self.h)
        return {"forward_ms": ms[0], "backward_ms": ms[1]}

    def close(self):
        if getattr(self, "h", None) is not None:
            load_library().pic_track_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # noqa: BLE001
            pass


def wake_polarization(tracker, E0, kp, x0, u0, s0):
    """Final polarization P (float64 tensor of 3) as a differentiable function
    of the torch scalars E0, kp and the (n, 3) tensors x0, u0, s0; the
    backward pass is the library's adjoint (pic_track_backward)."""
    import torch

    class _Fn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, e0, k, x, u, s):
            arrs = [t.detach().cpu().double().numpy() for t in (x, u, s)]
            P = tracker.forward(float(e0), float(k), *arrs)
            ctx.args = (float(e0), float(k), arrs)
            ctx.generation = tracker.generation
            ctx.devices = [t.device for t in (e0, k, x, u, s)]
            return torch.tensor(P, dtype=torch.float64, device=x.device)

        @staticmethod
        def backward(ctx, gP):
            if tracker.generation != ctx.generation:
                # another forward ran on this tracker since: recompute this one
                e0, k, arrs = ctx.args
                tracker.forward(e0, k, *arrs)
            gth, gx, gu, gs = tracker.backward(gP.detach().cpu().double().numpy())
            dv = ctx.devices
            return (torch.tensor(gth[0], dtype=torch.float64, device=dv[0]),
                    torch.tensor(gth[1], dtype=torch.float64, device=dv[1]),
                    torch.from_numpy(gx).to(dv[2]), torch.from_numpy(gu).to(dv[3]),
                    torch.from_numpy(gs).to(dv[4]))

    return _Fn.apply(E0, kp, x0, u0, s0)


# ---------------------------------------------------------------- batches

def _batch_check(code, b):
    if code != PIC_OK:
        msg = load_library().pic_batch_last_error(b)
        raise PicError(code, msg.decode() if msg else "")


class Batch:
    """Independent 2D runs stepped together (pic_batch_*).  cfgs: list of
    Config; states: list of (particles, fields) as for Simulation."""

    def __init__(self, cfgs, states, autotune=False, device=0):
        lib = load_library()
        n = len(cfgs)
        self.nruns = n
        self.cfgs = list(cfgs)
        carr = (Config * n)(*cfgs)
        keep = []
        sarr = (State * n)(*[_make_state(p, f, keep) for p, f in states])
        self.counts = [[len(p) if p is not None else 0 for p in parts] for parts, _ in states]
        self._mem = _TorchMemory(device)
        h = ctypes.c_void_p()
        _batch_check(lib.pic_batch_init(n, carr, sarr, 1 if autotune else 0, ctypes.byref(self._mem.allocator),
                                        self._mem.stream_handle, ctypes.byref(h)), None)
        self.h = h

    def step(self, n=1):
        _batch_check(load_library().pic_batch_step(self.h, int(n)), self.h)

    def polarization(self, run, species=-1, emin=-math.inf, emax=math.inf):
        P = np.zeros(3)
        N = ctypes.c_int64()
        _batch_check(load_library().pic_batch_polarization(self.h, int(run), int(species), float(emin), float(emax),
                                                           _dptr(P), ctypes.byref(N)), self.h)
        return P, int(N.value)

    def fields(self, run, names=FIELD_NAMES[:9]):
        c = self.cfgs[run]
        shape = (1, c.n[1], c.n[0])
        mask = 0
        for nm in names:
            mask |= 1 << FIELD_NAMES.index(nm)
        order = [nm for nm in FIELD_NAMES if nm in names]
        out = np.empty(len(order) * shape[1] * shape[2])
        _batch_check(load_library().pic_batch_fields(self.h, int(run), mask, _dptr(out), out.size), self.h)
        arr = out.reshape((len(order),) + shape)
        return {nm: arr[i] for i, nm in enumerate(order)}

    def particles(self, run, species):
        count = self.counts[run][species]
        out = np.empty((count, 11))
        n = ctypes.c_int64()
        _batch_check(load_library().pic_batch_particles(self.h, int(run), int(species), _dptr(out), out.size,
                                                        ctypes.byref(n)), self.h)
        return out[: n.value]

    def info(self, run):
        out = (ctypes.c_int64 * 4)()
        _batch_check(load_library().pic_batch_info(self.h, int(run), out), self.h)
        return {"tile": (out[0], out[1]), "particles": out[2], "cells": out[3]}

    def tuning(self):
        """None if nothing was tuned, else a dict: candidates (tile edges),
        share_ns ((nruns, ncand) ns per particle-step of each run's tiles over
        the push's workgroups, 0 where not tried), kernel_ms (push launch per
        uniform candidate) and mixed_ms (push launch with per-run tiles, 0 if
        not tried)."""
        nc = ctypes.c_int32()
        cands = (ctypes.c_int32 * 16)()
        ns = np.zeros(self.nruns * 16)
        kms = np.zeros(17)
        _batch_check(load_library().pic_batch_tuning(self.h, cands, _dptr(ns), _dptr(kms), 16, ctypes.byref(nc)),
                     self.h)
        n = nc.value
        if n == 0:
            return None
        return {"candidates": list(cands[:n]), "share_ns": ns[: self.nruns * n].reshape(self.nruns, n),
                "kernel_ms": kms[:n].copy(), "mixed_ms": float(kms[n])}

    def stats(self):
        out = (ctypes.c_int64 * 7)()
        _batch_check(load_library().pic_batch_stats(self.h, out, 7), self.h)
        return {"steps": out[0], "moved": out[1], "overflow": out[2], "repacks": out[3],
                "particles": out[4], "push_workgroups": out[5], "tiles": out[6]}

    def timing(self, enable=True, push_only=False):
        _batch_check(load_library().pic_batch_timing(self.h, _timing_mode(enable, push_only)), self.h)

    def timing_read(self):
        ms = np.zeros(4)
        n = (ctypes.c_int64 * 4)()
        _batch_check(load_library().pic_batch_timing_read(self.h, _dptr(ms), n, 4), self.h)
        return {nm: (ms[i], n[i]) for i, nm in enumerate(TIMER_NAMES)}

    def close(self):
        if getattr(self, "h", None) is not None:
            load_library().pic_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # noqa: BLE001
            pass
