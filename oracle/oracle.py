"""ctypes binding of the FP64 C oracle (lks_oracle.c).

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline timing).  Numpy
arrays in, numpy arrays out; layout [Q][ny][nx] / [k][ny][nx], x fastest.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lks_oracle.c")
_LIB = os.path.join(_HERE, "liblks_oracle.so")
NSUMS = 8

_lib = None


def build(force=True):
    """Compile the oracle with gcc (-O2, IEEE semantics, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-ffp-contract=off", "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC, "-lm"]
    if force or not os.path.exists(_LIB):
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int),
                ("tau", ctypes.c_double), ("mu", ctypes.c_double), ("dt", ctypes.c_double),
                ("dx", ctypes.c_double), ("mask", ctypes.c_uint), ("thr", ctypes.c_double * 8)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.orc_lattice.argtypes = [ctypes.c_int, P, P, P]
        lib.orc_equilibrium.argtypes = [ctypes.c_int, ctypes.c_long, P, P, P, P, P]
        lib.orc_moments.argtypes = [ctypes.c_int, ctypes.c_long, P, P]
        lib.orc_sensors.argtypes = [ctypes.c_int, ctypes.c_long, P, P]
        lib.orc_sensors.restype = ctypes.c_long
        lib.orc_d2q9_step.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, P, P, P, P, P,
                                      P, P, ctypes.c_uint, P]
        lib.orc_d2q9_step.restype = ctypes.c_long
        lib.orc_d2q25_step.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_int, P, P, P, P, P, P, ctypes.c_uint, P]
        lib.orc_d2q25_step.restype = ctypes.c_long
        lib.orc_run.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, P, P, P, P, P, P,
                                ctypes.c_int]
        lib.orc_run.restype = ctypes.c_long
        lib.orc_ext_sensors.argtypes = [ctypes.c_int, ctypes.c_long, P, ctypes.c_double, P]
        D = ctypes.c_double
        lib.orc_ddf_equilibrium.argtypes = [ctypes.c_long, P, P, P, P, D, P]
        lib.orc_ddf_moments.argtypes = [ctypes.c_long, P, D, P, P]
        lib.orc_ddf_step.argtypes = [ctypes.c_int, ctypes.c_int, D, D, D, D, D, ctypes.c_int,
                                     ctypes.c_int, P, P, P, P, P, P, ctypes.c_uint, P]
        lib.orc_ddf_step.restype = ctypes.c_long
        lib.orc_ddf_run.argtypes = [ctypes.c_int, ctypes.c_int, D, D, D, D, D, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, P, P, P, P, P, ctypes.c_uint, P,
                                    ctypes.c_int]
        lib.orc_ddf_run.restype = ctypes.c_long
        lib.orc_ddf_ext_sensors.argtypes = [ctypes.c_long, P, D, D, D, P]
        lib.orc_num_ext.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def lattice(q):
    """(vx, vy, w) of the D2Q9 (q=9) or GH5xGH5 D2Q25 (q=25) velocity set."""
    vx, vy, w = (np.zeros(q) for _ in range(3))
    if _load().orc_lattice(q, _p(vx), _p(vy), _p(w)) != q:
        raise ValueError(q)
    return vx, vy, w


def equilibrium(q, rho, ux, uy, T=None):
    """Grad-Hermite equilibrium populations [Q, *shape] of the fields."""
    rho = _f64(rho)
    shape = rho.shape
    n = rho.size
    out = np.empty((q,) + shape)
    _load().orc_equilibrium(q, n, _p(rho), _p(_f64(ux)), _p(_f64(uy)),
                            _p(None if T is None else _f64(T)), _p(out))
    return out


def moments(q, f):
    """rho, ux, uy, T [4, *shape] of populations f [Q, *shape]."""
    f = _f64(f)
    out = np.empty((4,) + f.shape[1:])
    _load().orc_moments(q, f[0].size, _p(f), _p(out))
    return out


def sensors(q, f):
    """(S_KL, S_NEQ, S_PI, S_Q) [4, *shape] of populations f, equilibrium from
    their own moments; also returns the number of positivity-fault cells."""
    f = _f64(f)
    out = np.empty((4,) + f.shape[1:])
    nf = _load().orc_sensors(q, f[0].size, _p(f), _p(out))
    return out, int(nf)


# extended sensor planes, in the order orc_ext_sensors writes them
EXT_NAMES = ("kn", "hr", "sigma_h", "sigma_hkl", "alpha", "shear", "qh", "qf", "comp", "strain")


def ext_sensors(q, f, par):
    """The extended sensors [len(EXT_NAMES), *shape] of populations f (the
    pre-collision state), equilibrium from their own moments; par = tau on
    D2Q9, mu on D2Q25."""
    f = _f64(f)
    lib = _load()
    assert lib.orc_num_ext() == len(EXT_NAMES)
    out = np.empty((len(EXT_NAMES),) + f.shape[1:])
    if lib.orc_ext_sensors(q, f[0].size, _p(f), float(par), _p(out)) != 0:
        raise ValueError(q)
    return out


# ---- D2Q25 double distribution (f, g) with the quasi-equilibrium collision
def cv_of(gamma):
    """Specific heat at constant volume C_v = R/(gamma - 1), R = 1."""
    return 1.0 / (gamma - 1.0)


def ddf_equilibrium(rho, ux, uy, T, gamma=1.4):
    """(f^eq, g^eq) [50, *shape] of the fields (f planes, then g planes)."""
    rho = _f64(rho)
    n = rho.size
    out = np.empty((50,) + rho.shape)
    _load().orc_ddf_equilibrium(n, _p(rho), _p(_f64(ux)), _p(_f64(uy)), _p(_f64(T)),
                                cv_of(gamma), _p(out))
    return out


def ddf_moments(f, gamma=1.4, qe=False):
    """rho, ux, uy, T [4, *shape] of a double-distribution state [50, *shape];
    with qe=True also (f^eq, g^eq, f*, g*) [100, *shape]."""
    f = _f64(f)
    n = f[0].size
    out = np.empty((4,) + f.shape[1:])
    q = np.empty((100,) + f.shape[1:]) if qe else None
    _load().orc_ddf_moments(n, _p(f), cv_of(gamma), _p(out), _p(q))
    return (out, q) if qe else out


def ddf_ext_sensors(f, mu, gamma=1.4, prandtl=0.71):
    """The extension sensors [len(EXT_NAMES), *shape] of a double-distribution
    state f [50, *shape] (g terms superposed, QE collision; COMP and STRAIN
    with the model's second viscosity -(gamma - 1) mu)."""
    f = _f64(f)
    n = f[0].size
    out = np.empty((len(EXT_NAMES),) + f.shape[1:])
    _load().orc_ddf_ext_sensors(n, _p(f), cv_of(gamma), float(mu), float(prandtl), _p(out))
    return out


def _thr5(thr):
    t = np.full(10, np.inf)
    if thr is not None:
        t[:] = np.asarray(thr, dtype=np.float64).reshape(10)
    return t


def ddf_step(f, mu, dt, dx, bc=(1, 1), gamma=1.4, prandtl=0.71, thr=None, mask=0):
    """One step of the double distribution.  Returns dict(f, mom, sens [5],
    flags, sums, faults)."""
    f = _f64(f)
    _, ny, nx = f.shape
    fo = np.empty_like(f)
    mom, sens = np.empty((4, ny, nx)), np.empty((5, ny, nx))
    flags = np.empty((ny, nx), np.uint8)
    sums = np.empty(NSUMS)
    nf = _load().orc_ddf_step(nx, ny, mu, prandtl, cv_of(gamma), dt, dx, bc[0], bc[1], _p(f), _p(fo),
                              _p(mom), _p(sens), _p(flags), _p(_thr5(thr)), mask, _p(sums))
    return dict(f=fo, mom=mom, sens=sens, flags=flags, sums=sums, faults=int(nf))


def ddf_run(f0, nsteps, mu, dt, dx, bc=(1, 1), gamma=1.4, prandtl=0.71, thr=None, mask=0,
            nthreads=0):
    """Run nsteps of the double distribution from f0 [50, ny, nx]."""
    f = _f64(f0).copy()
    _, ny, nx = f.shape
    mom, sens = np.empty((4, ny, nx)), np.empty((5, ny, nx))
    flags = np.empty((ny, nx), np.uint8)
    sums = np.zeros((max(nsteps, 1), NSUMS))
    nf = _load().orc_ddf_run(nx, ny, mu, prandtl, cv_of(gamma), dt, dx, bc[0], bc[1], nsteps, _p(f),
                             _p(mom), _p(sens), _p(flags), _p(_thr5(thr)), mask, _p(sums), nthreads)
    return dict(f=f, mom=mom, sens=sens, flags=flags, sums=sums[:nsteps], faults=int(nf))


def _thr(thr):
    t = np.full(8, np.inf)
    if thr is not None:
        t[:] = np.asarray(thr, dtype=np.float64).reshape(8)
    return t


def d2q9_step(f, tau, thr=None, mask=0):
    """One D2Q9 LBGK step.  Returns dict(f, g, mom, sens, flags, sums, faults)."""
    f = _f64(f)
    _, ny, nx = f.shape
    fo, g = np.empty_like(f), np.empty_like(f)
    mom, sens = np.empty((4, ny, nx)), np.empty((4, ny, nx))
    flags = np.empty((ny, nx), np.uint8)
    sums = np.empty(NSUMS)
    t = _thr(thr)
    nf = _load().orc_d2q9_step(nx, ny, tau, _p(f), _p(fo), _p(g), _p(mom), _p(sens), _p(flags),
                               _p(t), mask, _p(sums))
    return dict(f=fo, g=g, mom=mom, sens=sens, flags=flags, sums=sums, faults=int(nf))


def d2q25_step(f, mu, dt, dx, bc=(1, 1), thr=None, mask=0):
    """One D2Q25 finite-volume step.  bc = (bc_x, bc_y), 0 periodic, 1 outflow."""
    f = _f64(f)
    _, ny, nx = f.shape
    fo = np.empty_like(f)
    mom, sens = np.empty((4, ny, nx)), np.empty((4, ny, nx))
    flags = np.empty((ny, nx), np.uint8)
    sums = np.empty(NSUMS)
    t = _thr(thr)
    nf = _load().orc_d2q25_step(nx, ny, mu, dt, dx, bc[0], bc[1], _p(f), _p(fo), _p(mom),
                                _p(sens), _p(flags), _p(t), mask, _p(sums))
    return dict(f=fo, mom=mom, sens=sens, flags=flags, sums=sums, faults=int(nf))


def run(q, f0, nsteps, tau=0.0, mu=0.0, dt=0.0, dx=1.0, bc=(0, 0), thr=None, mask=0,
        nthreads=0):
    """Run nsteps from populations f0.  Returns dict(f, mom, sens, flags, sums,
    flag_counts, faults) with the last step's fields and per-step sums."""
    f = _f64(f0).copy()
    _, ny, nx = f.shape
    p = _Params(lattice=q, nx=nx, ny=ny, bc_x=bc[0], bc_y=bc[1], tau=tau, mu=mu, dt=dt, dx=dx,
                mask=mask)
    p.thr[:] = list(_thr(thr))
    mom, sens = np.empty((4, ny, nx)), np.empty((4, ny, nx))
    flags = np.empty((ny, nx), np.uint8)
    sums = np.zeros((max(nsteps, 1), NSUMS))
    counts = np.zeros((max(nsteps, 1), 3), np.int64)
    nf = _load().orc_run(ctypes.byref(p), nsteps, _p(f), _p(mom), _p(sens), _p(flags), _p(sums),
                         _p(counts), nthreads)
    return dict(f=f, mom=mom, sens=sens, flags=flags, sums=sums[:nsteps],
                flag_counts=counts[:nsteps], faults=int(nf))


def flags_from_sensors(sens, thr, mask, fault=None):
    """Flag map from a sensor stack [4, ...] (numpy, the same rule as the C
    oracle: per enabled sensor (s > t1) + (s > t2), max over sensors, fault
    cells 2 | 0x80)."""
    thr = np.asarray(thr, dtype=np.float64).reshape(4, 2)
    level = np.zeros(sens.shape[1:], np.uint8)
    for k in range(4):
        if mask & (1 << k):
            lk = (sens[k] > thr[k, 0]).astype(np.uint8) + (sens[k] > thr[k, 1]).astype(np.uint8)
            level = np.maximum(level, lk)
    if fault is not None:
        level = np.where(fault, np.uint8(0x82), level)
    return level
