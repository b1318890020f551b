"""Thin Python binding of liblks.so (ctypes): argument marshalling only.

Every step of the kinetic path runs in the library's HIP kernels; PyTorch
provides the device memory (caller-owned buffers) and the stream.  There is no
CPU fallback: if the library is missing or no GPU is present, calls raise.
Names follow include/lks.h.
"""
import ctypes
import math
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblks.so")

D2Q9, D2Q25 = 9, 25
F64, F32, BF16, F16 = 0, 1, 2, 3
PERIODIC, OUTFLOW = 0, 1
S_KL, S_NEQ, S_PI, S_Q, S_QE = 1, 2, 4, 8, 16
MODEL_BGK, MODEL_DDF = 0, 1
MODELS = {"bgk": MODEL_BGK, "ddf": MODEL_DDF}
LAYOUT_PLANES, LAYOUT_ROWS = 0, 1
LAYOUTS = {"planes": LAYOUT_PLANES, "rows": LAYOUT_ROWS}
NSUMS = 8
# extension sensors (bit k of ext_mask; flag_mask bit 8 + k), plane order
EXT_NAMES = ("kn", "hr", "sigma_h", "sigma_hkl", "alpha", "shear", "qh", "qf", "comp", "strain")
MAX_EXT = len(EXT_NAMES)


def flag_x(k):
    """flag_mask bit of extension sensor k (an index or a name)."""
    k = EXT_NAMES.index(k) if isinstance(k, str) else int(k)
    return 1 << (8 + k)


def ext_mask_of(ext):
    """ext_mask from an int mask or an iterable of names / indices."""
    if ext is None:
        return 0
    if isinstance(ext, int):
        return ext
    m = 0
    for k in ext:
        m |= 1 << (EXT_NAMES.index(k) if isinstance(k, str) else int(k))
    return m
STATUS = {0: "LKS_OK", 1: "LKS_EINVAL", 2: "LKS_ESTATE", 3: "LKS_EHIP", 4: "LKS_ENONPOS",
          5: "LKS_ENAN", 6: "LKS_EUNSUPPORTED"}
DTYPES = {"f64": F64, "f32": F32, "bf16": BF16, "f16": F16}
_TORCH_STORE = {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16, F16: torch.float16}


class LksError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
                ("tau", ctypes.c_double), ("mu", ctypes.c_double), ("dt", ctypes.c_double),
                ("dx", ctypes.c_double), ("rho0", ctypes.c_double),
                ("flag_mask", ctypes.c_uint32), ("launch_rows", ctypes.c_int32),
                ("thr", (ctypes.c_double * 2) * 4), ("max_steps", ctypes.c_int32),
                ("launch_vec", ctypes.c_int32), ("ext_mask", ctypes.c_uint32),
                ("ext_reserved", ctypes.c_int32), ("thr_ext", (ctypes.c_double * 2) * MAX_EXT),
                ("model", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("prandtl", ctypes.c_double),
                ("thr_qe", ctypes.c_double * 2), ("launch_nt", ctypes.c_int32),
                ("launch_steps", ctypes.c_int32)]


class Box(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_int32), ("y0", ctypes.c_int32), ("x1", ctypes.c_int32),
                ("y1", ctypes.c_int32)]


MACRO_NAMES = ("tau", "c", "s", "e", "qh", "qf", "qnsf")


class Transport(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("lambda_", ctypes.c_double), ("kappa", ctypes.c_double),
                ("per_rho", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Buffers(ctypes.Structure):
    _fields_ = [("pop", ctypes.c_void_p * 2), ("sensors", ctypes.c_void_p),
                ("flags", ctypes.c_void_p), ("sums", ctypes.c_void_p),
                ("scratch", ctypes.c_void_p), ("scratch_bytes", ctypes.c_size_t)]


_lib = None


def lib():
    """The loaded liblks.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run python -m paper_2603_13618_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        sig = {
            "lks_scratch_bytes": ([ctypes.POINTER(Config)], ctypes.c_size_t),
            "lks_num_sensors": ([I32], I32),
            "lks_sensor_planes": ([ctypes.POINTER(Config)], I32),
            "lks_create": ([ctypes.POINTER(Config), ctypes.POINTER(Buffers), P, ctypes.POINTER(P)], I32),
            "lks_init_equilibrium": ([P, P, P, P, P], I32),
            "lks_restore": ([P, I32, I64], I32),
            "lks_step": ([P, I32, I32], I32),
            "lks_step_from": ([P, P, P], I32),
            "lks_step_noalloc": ([ctypes.POINTER(Config), ctypes.POINTER(Buffers), P, I32, I64, I32, I32,
                                  ctypes.POINTER(I32)], I32),
            "lks_current": ([P, ctypes.POINTER(I32), ctypes.POINTER(I64)], I32),
            "lks_moments": ([P, P, P, P, P], I32),
            "lks_read_host": ([P, I32, P, ctypes.c_size_t], I32),
            "lks_check": ([P, ctypes.POINTER(I64)], I32),
            "lks_adjoint_seed_kl": ([P, P, P], I32),
            "lks_adjoint_step": ([P, P, P, P], I32),
            "lks_adjoint_init": ([P, P, P, P, P, P, P], I32),
            "lks_destroy": ([P], I32),
            "lks_status_str": ([I32], ctypes.c_char_p),
            "lks_last_error": ([P], ctypes.c_char_p),
            "lks_copy_probe": ([P, P, ctypes.c_size_t, P], I32),
            "lks_tag_buffer": ([P, I32, P, P], I32),
            "lks_macro_sensors": ([P, P, P, P, P, ctypes.POINTER(Transport), ctypes.c_uint32, P], I32),
            "lks_tag_tiles": ([P, P, I32, I32, P], I32),
            "lks_cluster": ([P, I32, I32, I32, ctypes.c_double, I32, ctypes.POINTER(Box), I32,
                             ctypes.POINTER(I32)], I32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def same_layout(t, ref):
    """True if tensor t holds a state exactly as ref does: shape, dtype,
    device, element strides (those of dimensions of length 1 carry no
    information) and no storage offset."""
    strides = all(a == b for a, b, n in zip(t.stride(), ref.stride(), ref.shape) if n > 1)
    return (tuple(t.shape) == tuple(ref.shape) and t.dtype == ref.dtype and t.device == ref.device
            and strides and t.storage_offset() == 0)


def _stream_handle(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def make_config(lattice=D2Q9, nx=64, ny=64, dtype=F32, tau=0.6, mu=0.0, dt=0.0, dx=1.0,
                bc=(PERIODIC, PERIODIC), rho0=1.0, thr=None, flag_mask=0, max_steps=1,
                launch_rows=0, launch_vec=0, ext=None, thr_ext=None, model=MODEL_BGK, gamma=1.4,
                prandtl=0.71, thr_qe=None, layout=LAYOUT_PLANES, launch_nt=0, launch_steps=0):
    c = Config()
    c.lattice, c.nx, c.ny = lattice, nx, ny
    c.dtype = DTYPES[dtype] if isinstance(dtype, str) else dtype
    c.bc_x, c.bc_y = bc
    c.tau, c.mu, c.dt, c.dx, c.rho0 = tau, mu, dt, dx, rho0
    c.flag_mask = flag_mask
    c.launch_rows = launch_rows
    t = np.full((4, 2), math.inf) if thr is None else np.asarray(thr, np.float64).reshape(4, 2)
    for s in range(4):
        c.thr[s][0], c.thr[s][1] = float(t[s, 0]), float(t[s, 1])
    c.max_steps = max_steps
    c.launch_vec = launch_vec
    c.ext_mask = ext_mask_of(ext)
    c.ext_reserved = 0
    te = (np.full((MAX_EXT, 2), math.inf) if thr_ext is None
          else np.asarray(thr_ext, np.float64).reshape(MAX_EXT, 2))
    for k in range(MAX_EXT):
        c.thr_ext[k][0], c.thr_ext[k][1] = float(te[k, 0]), float(te[k, 1])
    c.model = MODELS[model] if isinstance(model, str) else model
    c.layout = LAYOUTS[layout] if isinstance(layout, str) else layout
    c.launch_nt, c.launch_steps = launch_nt, launch_steps
    c.gamma, c.prandtl = gamma, prandtl
    tq = (math.inf, math.inf) if thr_qe is None else tuple(float(v) for v in thr_qe)
    c.thr_qe[0], c.thr_qe[1] = tq
    return c


def scratch_bytes(cfg):
    return int(lib().lks_scratch_bytes(ctypes.byref(cfg)))


def _check(status, ctx=None):
    if status != 0:
        msg = lib().lks_last_error(ctx).decode()
        raise LksError(status, msg)


class Lattice:
    """One simulation context with torch-owned device buffers.

    Attributes: pop (2 tensors [Q, ny, nx]: views of the state buffers, which
    are [ny, Q, nx] with layout "rows" (default; the faster one for D2Q9
    FP32/FP64 storage and never slower) and [Q, ny, nx] with layout "planes";
    new_state() makes another), sensors [nsens, ny, nx] (the
    base sensors, then one plane per extension sensor in ext, in EXT_NAMES
    order), flags [ny, nx] uint8, sums [max_steps, 8] float64.
    ext: extension sensors (names from EXT_NAMES, indices or a bit mask);
    thr_ext: [MAX_EXT, 2] thresholds, used for sensors whose flag_x bit is in
    flag_mask.
    model: "bgk" (default) or, on D2Q25, "ddf" -- the (f, g) double
    distribution with the quasi-equilibrium collision (gamma, prandtl; pop
    then holds 50 planes, f then g, and sensors 5 planes, the fifth S_QE with
    thresholds thr_qe and flag bit S_QE).
    launch_steps: 2 runs two fused D2Q9 steps per launch (no extension
    sensors; pairs need max_steps >= 2); state, sensors, flags and fault
    counts are the same bits (the per-step sums agree to FP64 rounding), and
    `state` follows the buffer that holds the current state.
    """

    def __init__(self, lattice=D2Q9, nx=64, ny=64, dtype="f32", tau=0.6, mu=0.0, dt=0.0, dx=1.0,
                 bc=(PERIODIC, PERIODIC), rho0=1.0, thr=None, flag_mask=0, max_steps=1,
                 launch_rows=0, launch_vec=0, ext=None, thr_ext=None, model=MODEL_BGK, gamma=1.4,
                 prandtl=0.71, thr_qe=None, layout=LAYOUT_ROWS, launch_nt=0, launch_steps=0,
                 device="cuda"):
        self.device = torch.device(device)
        self.cfg = make_config(lattice, nx, ny, dtype, tau, mu, dt, dx, bc, rho0, thr, flag_mask,
                               max_steps, launch_rows, launch_vec, ext, thr_ext, model, gamma,
                               prandtl, thr_qe, layout, launch_nt, launch_steps)
        self.layout = self.cfg.layout
        self.model = self.cfg.model
        self.Q = 50 if self.model == MODEL_DDF else lattice
        self.nx, self.ny = nx, ny
        self.dtype = self.cfg.dtype
        nsens = int(lib().lks_sensor_planes(ctypes.byref(self.cfg))) or \
            int(lib().lks_num_sensors(lattice))
        self.ext_mask = self.cfg.ext_mask
        sdt = torch.float64 if self.dtype == F64 else torch.float32
        tdt = _TORCH_STORE[self.dtype]
        dev = self.device
        self.pop = [self._alloc_state(tdt, dev, torch.zeros) for _ in range(2)]
        self.sensors = torch.zeros((nsens, ny, nx), dtype=sdt, device=dev)
        self.flags = torch.zeros((ny, nx), dtype=torch.uint8, device=dev)
        self.sums = torch.zeros((max_steps, NSUMS), dtype=torch.float64, device=dev)
        nsb = scratch_bytes(self.cfg)
        if nsb == 0:
            raise LksError(1, "invalid configuration")
        self.scratch = torch.zeros(nsb, dtype=torch.uint8, device=dev)
        self.buf = Buffers()
        self.buf.pop[0] = self.pop[0].data_ptr()
        self.buf.pop[1] = self.pop[1].data_ptr()
        self.buf.sensors = self.sensors.data_ptr()
        self.buf.flags = self.flags.data_ptr()
        self.buf.sums = self.sums.data_ptr()
        self.buf.scratch = self.scratch.data_ptr()
        self.buf.scratch_bytes = nsb
        self.ctx = ctypes.c_void_p()
        st = lib().lks_create(ctypes.byref(self.cfg), ctypes.byref(self.buf),
                              _stream_handle(dev), ctypes.byref(self.ctx))
        _check(st, None)

    def _alloc_state(self, tdt, dev, make=torch.empty):
        if self.layout == LAYOUT_ROWS:
            return make((self.ny, self.Q, self.nx), dtype=tdt, device=dev).permute(1, 0, 2)
        return make((self.Q, self.ny, self.nx), dtype=tdt, device=dev)

    def new_state(self):
        """An uninitialised state tensor [Q, ny, nx] in this context's layout."""
        return self._alloc_state(self.pop[0].dtype, self.device)

    def _state_arg(self, t, what):
        if not same_layout(t, self.pop[0]):
            raise ValueError(f"{what} must be a [Q, ny, nx] {self.pop[0].dtype} state in this "
                             f"context's layout (strides {self.pop[0].stride()}): use new_state()")
        return _ptr(t)

    def macro_sensors(self, rho, ux, uy, T=None, mu=0.0, lam=0.0, kappa=0.0, per_rho=False,
                      which=MACRO_NAMES, out=None):
        """The macroscopic class-1 sensors (central differences) of FP64 device
        fields [ny, nx]: dict name -> plane of `out` ([len(which), ny, nx] FP64)."""
        mask = 0
        for n in which:
            mask |= 1 << MACRO_NAMES.index(n)
        names = [n for n in MACRO_NAMES if mask & (1 << MACRO_NAMES.index(n))]
        if out is None:
            out = torch.empty((len(names), self.ny, self.nx), dtype=torch.float64, device=self.device)
        tr = Transport(float(mu), float(lam), float(kappa), 1 if per_rho else 0, 0)
        _check(lib().lks_macro_sensors(self.ctx, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T),
                                       ctypes.byref(tr), mask, _ptr(out)), self.ctx)
        return {n: out[k] for k, n in enumerate(names)}

    def tag_buffer(self, b=2, flags=None, out=None):
        """Buffer layer of b cells around the tagged cells of `flags` (default:
        this context's flag map): uint8 levels [ny, nx] on the device."""
        flags = self.flags if flags is None else flags
        out = torch.empty((self.ny, self.nx), dtype=torch.uint8, device=self.device) if out is None else out
        _check(lib().lks_tag_buffer(self.ctx, int(b), _ptr(flags), _ptr(out)), self.ctx)
        return out

    def tag_tiles(self, levels, level=1, ts=8, out=None):
        """Cells at level >= `level` per ts x ts tile: int32 [ceil(ny/ts), ceil(nx/ts)]."""
        shape = (-(-self.ny // ts), -(-self.nx // ts))
        out = torch.empty(shape, dtype=torch.int32, device=self.device) if out is None else out
        _check(lib().lks_tag_tiles(self.ctx, _ptr(levels), int(level), int(ts), _ptr(out)), self.ctx)
        return out

    def ext(self, name):
        """The sensor plane of extension sensor `name` (must be in ext)."""
        k = EXT_NAMES.index(name)
        if not self.ext_mask & (1 << k):
            raise KeyError(name)
        base = 5 if self.model == MODEL_DDF else int(lib().lks_num_sensors(self.cfg.lattice))
        return self.sensors[base + bin(self.ext_mask & ((1 << k) - 1)).count("1")]

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx and _lib is not None:
            _lib.lks_destroy(ctx)
            self.ctx = None

    def _field(self, a):
        if a is None:
            return None
        t = torch.as_tensor(a, dtype=torch.float64)
        return t.to(self.device).contiguous()

    def init(self, rho, ux, uy, T=None):
        """Equilibrium initial state of FP64 fields [ny, nx] (numpy or torch)."""
        self._init_fields = [self._field(a) for a in (rho, ux, uy, T)]
        f = self._init_fields
        _check(lib().lks_init_equilibrium(self.ctx, _ptr(f[0]), _ptr(f[1]), _ptr(f[2]),
                                          _ptr(f[3])), self.ctx)

    def restore(self, state, steps_done=0):
        """Copy a state [Q, ny, nx] (storage dtype) into pop[0] and resume from it."""
        self.pop[0].copy_(torch.as_tensor(state).to(self.device, self.pop[0].dtype))
        _check(lib().lks_restore(self.ctx, 0, int(steps_done)), self.ctx)

    def step(self, nsteps=1, fused=True):
        _check(lib().lks_step(self.ctx, int(nsteps), 1 if fused else 0), self.ctx)

    def step_from(self, src, dst):
        """One fused step from the state tensor src into dst (step count unchanged)."""
        _check(lib().lks_step_from(self.ctx, self._state_arg(src, "src"),
                                   self._state_arg(dst, "dst")), self.ctx)

    def current(self):
        i, n = ctypes.c_int32(), ctypes.c_int64()
        _check(lib().lks_current(self.ctx, ctypes.byref(i), ctypes.byref(n)), self.ctx)
        return i.value, n.value

    @property
    def state(self):
        return self.pop[self.current()[0]]

    def moments(self):
        """(rho, ux, uy, T) FP64 device tensors of the current state."""
        out = [torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
               for _ in range(4)]
        _check(lib().lks_moments(self.ctx, *[_ptr(t) for t in out]), self.ctx)
        return out

    def check(self):
        """Synchronise; returns the positivity-fault count (raises on NaN sums)."""
        n = ctypes.c_int64()
        st = lib().lks_check(self.ctx, ctypes.byref(n))
        if st not in (0, 4):
            _check(st, self.ctx)
        return n.value

    def read_host(self, what):
        """Synchronous copy to a numpy array through lks_read_host (what 0..3)."""
        src = [self.state, self.sensors, self.flags, self.sums][what]
        rows = what == 0 and self.layout == LAYOUT_ROWS
        shape = (self.ny, self.Q, self.nx) if rows else tuple(src.shape)
        if src.dtype == torch.bfloat16:
            out = np.empty(shape, np.uint16)
        else:
            out = np.empty(shape, {torch.float64: np.float64, torch.float32: np.float32,
                                   torch.float16: np.float16, torch.uint8: np.uint8}[src.dtype])
        _check(lib().lks_read_host(self.ctx, what, out.ctypes.data_as(ctypes.c_void_p),
                                   out.nbytes), self.ctx)
        return out.transpose(1, 0, 2) if rows else out

    # ---- adjoint (D2Q9) ----
    def adjoint_seed_kl(self, pop_prev, lam_out):
        _check(lib().lks_adjoint_seed_kl(self.ctx, self._state_arg(pop_prev, "pop_prev"),
                                         self._state_arg(lam_out, "lam_out")), self.ctx)

    def adjoint_step(self, pop_prev, lam_in, lam_out):
        _check(lib().lks_adjoint_step(self.ctx, self._state_arg(pop_prev, "pop_prev"),
                                      self._state_arg(lam_in, "lam_in"),
                                      self._state_arg(lam_out, "lam_out")), self.ctx)

    def adjoint_init(self, rho0, ux0, uy0, lam0, gux, guy):
        _check(lib().lks_adjoint_init(self.ctx, _ptr(rho0), _ptr(ux0), _ptr(uy0),
                                      self._state_arg(lam0, "lam0"),
                                      _ptr(gux), _ptr(guy)), self.ctx)


def cluster(counts, nx, ny, ts, eff=0.98, min_tiles=1, max_boxes=None):
    """Berger-Rigoutsos patches of a host tile-count array (as written by
    Lattice.tag_tiles): list of (x0, y0, x1, y1) cell boxes, half-open."""
    c = np.ascontiguousarray(counts, dtype=np.int32)
    if max_boxes is None:
        max_boxes = max(int(np.count_nonzero(c)), 1)       # at most one box per tagged tile
    boxes = (Box * max_boxes)()
    n = ctypes.c_int32()
    st = lib().lks_cluster(c.ctypes.data_as(ctypes.c_void_p), int(nx), int(ny), int(ts), float(eff),
                           int(min_tiles), boxes, int(max_boxes), ctypes.byref(n))
    if st != 0:
        raise LksError(st, f"lks_cluster needs {n.value} boxes (room for {max_boxes})"
                       if n.value > max_boxes else "invalid clustering arguments")
    return [(b.x0, b.y0, b.x1, b.y1) for b in boxes[: n.value]]


NOALLOC_SCRATCH_BYTES = 16 << 20      # LKS_NOALLOC_SCRATCH_BYTES


def step_noalloc(cfg, pop, sensors, flags, sums, pop_index=0, steps_done=0, nsteps=1, fused=True):
    """lks_step_noalloc: nsteps steps of the state in pop[pop_index] (a state
    reached after steps_done steps) with the library's own device scratch,
    on torch's current stream; pop is a pair of state tensors, sensors, flags
    and sums as a Lattice of cfg holds them.  Returns the index of the buffer
    that holds the new state."""
    buf = Buffers()
    buf.pop[0], buf.pop[1] = pop[0].data_ptr(), pop[1].data_ptr()
    buf.sensors, buf.flags, buf.sums = sensors.data_ptr(), flags.data_ptr(), sums.data_ptr()
    buf.scratch, buf.scratch_bytes = None, 0
    out = ctypes.c_int32(-1)
    _check(lib().lks_step_noalloc(ctypes.byref(cfg), ctypes.byref(buf), _stream_handle(pop[0].device),
                                  int(pop_index), int(steps_done), int(nsteps), 1 if fused else 0,
                                  ctypes.byref(out)))
    return out.value


def copy_probe(dst, src):
    """Device copy of src into dst (same byte size) with the library's copy kernel."""
    nbytes = src.numel() * src.element_size()
    _check(lib().lks_copy_probe(_ptr(dst), _ptr(src), nbytes, _stream_handle(src.device)))

