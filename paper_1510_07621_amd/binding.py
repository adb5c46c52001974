"""Python binding of libp3m.so: the same entry points, argument marshalling only.

Every computation runs in the HIP library; this module checks tensor shapes,
dtypes and devices, passes raw device pointers and the current PyTorch (HIP)
stream, and turns status codes into exceptions. PyTorch supplies device
memory and streams. Importing this module loads the library and raises
``RuntimeError`` if it has not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch  # loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
# P3M_LIBRARY selects another build of the same library (e.g. a debug build).
LIB_PATH = os.environ.get("P3M_LIBRARY") or os.path.join(_HERE, "libp3m.so")

P3M_OK, P3M_EINVAL, P3M_ENOMEM, P3M_EHIP, P3M_ERANGE, P3M_ESIZE = 0, -1, -2, -3, -4, -5
P3M_FP64, P3M_FP32 = 0, 1
STAGES = ("bin", "deposit", "fft", "interp", "pp", "react")


class P3MParams(ctypes.Structure):
    _fields_ = [
        ("grid_n", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("fd_order", ctypes.c_int32),
        ("deconv_power", ctypes.c_int32),
        ("box", ctypes.c_double),
        ("rs_cells", ctypes.c_double),
        ("cutoff_rs", ctypes.c_double),
        ("softening", ctypes.c_double),
        ("G", ctypes.c_double),
        ("adjoint", ctypes.c_int32),
        ("ewald_gridsize", ctypes.c_int32),
        ("pair_partials", ctypes.c_int32),
    ]


class P3MCosmology(ctypes.Structure):
    _fields_ = [("H0", ctypes.c_double), ("Omega_m", ctypes.c_double),
                ("Omega_L", ctypes.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run `python -m paper_1510_07621_amd.build` "
            "(the force path has no fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    sig = {
        "p3m_params_default": (ctypes.c_int, [ctypes.POINTER(P3MParams), i32, dbl]),
        "p3m_plan_create": (ctypes.c_int, [ctypes.POINTER(P3MParams), i64, vp,
                                           ctypes.POINTER(vp)]),
        "p3m_plan_destroy": (ctypes.c_int, [vp]),
        "p3m_plan_set_stream": (ctypes.c_int, [vp, vp]),
        "p3m_force": (ctypes.c_int, [vp, i64, vp, vp, dbl, vp, i32]),
        "pm_force": (ctypes.c_int, [vp, i64, vp, vp, dbl, vp, i32]),
        "pp_force": (ctypes.c_int, [vp, i64, vp, vp, dbl, vp, i32]),
        "p3m_pair_count": (ctypes.c_int, [vp, i64, vp, vp]),
        "pp_force_noalloc": (ctypes.c_int, [ctypes.POINTER(P3MParams), i64, vp, vp, dbl, vp,
                                            i32, vp]),
        "p3m_force_vjp": (ctypes.c_int, [vp, i64, vp, vp, dbl, vp, vp]),
        "pp_ewald_force": (ctypes.c_int, [vp, i64, vp, vp, dbl, vp, i32]),
        "p3m_ewald_correction": (ctypes.c_int, [vp, i64, vp, vp]),
        "p3m_power_spectrum": (ctypes.c_int, [vp, i64, vp, vp, dbl, i32, dbl, vp, vp, vp,
                                              vp]),
        "pm_force_vjp": (ctypes.c_int, [vp, i64, vp, vp, dbl, vp, vp]),
        "pp_force_vjp": (ctypes.c_int, [vp, i64, vp, vp, dbl, vp, vp]),
        "p3m_drift_vjp": (ctypes.c_int, [i64, vp, vp, vp, dbl, dbl, vp]),
        "p3m_kick": (ctypes.c_int, [i64, vp, vp, i32, dbl, vp]),
        "p3m_force_cell_order": (ctypes.c_int, [vp, i64, vp, vp, dbl, vp, i32, vp]),
        "p3m_kick_reorder": (ctypes.c_int, [i64, vp, vp, vp, vp, i32, vp, vp, dbl, vp, vp, vp,
                                            vp, vp]),
        "p3m_kick_drift": (ctypes.c_int, [i64, vp, vp, vp, i32, vp, dbl, dbl, dbl, dbl, vp]),
        "p3m_drift": (ctypes.c_int, [i64, vp, vp, vp, dbl, dbl, dbl, vp]),
        "p3m_set_timing": (ctypes.c_int, [vp, i32]),
        "p3m_stage_times": (ctypes.c_int, [vp, ctypes.POINTER(dbl), i32]),
        "p3m_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "p3m_stencil_rows": (i32, [i32, dbl, ctypes.POINTER(i32), i32]),
        "p3m_segment_rows": (i32, [i32, dbl, ctypes.POINTER(i32), i32]),
        "p3m_group_edge": (i32, [i64, i32]),
        "p3m_split_table": (i32, [dbl, dbl, ctypes.POINTER(ctypes.c_float), i32,
                                  ctypes.POINTER(dbl)]),
        "p3m_split_table64": (i32, [dbl, dbl, ctypes.POINTER(dbl), i32, ctypes.POINTER(dbl)]),
        "p3m_cosmo_age": (ctypes.c_int, [ctypes.POINTER(P3MCosmology), dbl,
                                         ctypes.POINTER(dbl)]),
        "p3m_cosmo_scale_factor": (ctypes.c_int, [ctypes.POINTER(P3MCosmology), dbl,
                                                  ctypes.POINTER(dbl)]),
        "p3m_cosmo_kick_drift": (ctypes.c_int, [ctypes.POINTER(P3MCosmology), dbl, dbl,
                                                ctypes.POINTER(dbl), ctypes.POINTER(dbl)]),
        "p3m_cosmo_kdk_step": (ctypes.c_int, [ctypes.POINTER(P3MCosmology), dbl, dbl,
                                              ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                              ctypes.POINTER(dbl), ctypes.POINTER(dbl)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def strerror(status: int) -> str:
    return _lib.p3m_strerror(status).decode()


def _check(status: int, what: str) -> None:
    if status == P3M_OK:
        return
    msg = f"{what}: {strerror(status)} (status {status})"
    if status in (P3M_EINVAL, P3M_ERANGE, P3M_ESIZE):
        raise ValueError(msg)
    raise RuntimeError(msg)


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def _vec3(t: torch.Tensor, name: str, dtype=torch.float64) -> int:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype or t.dim() != 2 or t.shape[0] != 3 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous (3, n) {dtype} tensor")
    return int(t.shape[1])


def _mass(mass, n):
    if mass is None or isinstance(mass, (int, float)):
        return None, float(1.0 if mass is None else mass)
    if (not isinstance(mass, torch.Tensor) or mass.device.type != "cuda" or
            mass.dtype != torch.float64 or mass.shape != (n,) or not mass.is_contiguous()):
        raise ValueError("mass must be a scalar or a contiguous (n,) float64 GPU tensor")
    return mass, 0.0


def stencil_rows(g: int, radius_cells: float):
    """Neighbour stencil rows (dx, dy, dz_lo, dz_hi) of a g^3-cell i-group."""
    n = _lib.p3m_stencil_rows(g, radius_cells, None, 0)
    _check(min(n, 0), "p3m_stencil_rows")
    buf = (ctypes.c_int32 * (4 * n))()
    _lib.p3m_stencil_rows(g, radius_cells, buf, n)
    return [tuple(buf[4 * k:4 * k + 4]) for k in range(n)]


def segment_rows(g: int, radius_cells: float):
    """The stencil cut into group segments (dx, dy, dz_lo, dz_hi, sign), sign
    the lexicographic sign of the segment's group offset (0: the group)."""
    n = _lib.p3m_segment_rows(g, radius_cells, None, 0)
    _check(min(n, 0), "p3m_segment_rows")
    buf = (ctypes.c_int32 * (4 * max(n, 1)))()
    _lib.p3m_segment_rows(g, radius_cells, buf, n)
    out = []
    for k in range(n):
        p = buf[4 * k]
        dx = ((p & 0xffff) ^ 0x8000) - 0x8000
        out.append((dx, p >> 16, buf[4 * k + 1], buf[4 * k + 2], buf[4 * k + 3]))
    return out


def group_edge(n: int, grid_n: int) -> int:
    return int(_lib.p3m_group_edge(n, grid_n))


def split_table(cutoff_rs: float, softening_rs: float = 0.0):
    """FP32 split-factor table of the pair sum: a (4, B + 1) float32 array of
    cubic coefficients c0..c3 per bin, and the map (variable, v0, v1): the
    variable is 0 for r / r_s, 1 for sqrt(r^2 + eps^2) / r_s, and the bins cut
    [v0, v1] evenly."""
    import numpy as np
    b = _lib.p3m_split_table(cutoff_rs, softening_rs, None, 0, None)
    _check(min(b, 0), "p3m_split_table")
    buf = (ctypes.c_float * (4 * (b + 1)))()
    m = (ctypes.c_double * 3)()
    _check(min(_lib.p3m_split_table(cutoff_rs, softening_rs, buf, 4 * (b + 1), m), 0),
           "p3m_split_table")
    tab = np.frombuffer(buf, dtype=np.float32).reshape(4, b + 1).copy()
    return tab, (int(m[0]), float(m[1]), float(m[2]))


def split_table64(cutoff_rs: float, softening_rs: float = 0.0):
    """FP64 split-factor table of the pair sum: a (7, B + 1) float64 array, row
    l the coefficient of t^l (t the position in the bin, 0..1) of each bin,
    and the map (variable, v0, v1, exact bins) as for split_table plus the
    leading bins evaluated exactly."""
    import numpy as np
    b = _lib.p3m_split_table64(cutoff_rs, softening_rs, None, 0, None)
    _check(min(b, 0), "p3m_split_table64")
    buf = (ctypes.c_double * (7 * (b + 1)))()
    m = (ctypes.c_double * 4)()
    _check(min(_lib.p3m_split_table64(cutoff_rs, softening_rs, buf, 7 * (b + 1), m), 0),
           "p3m_split_table64")
    tab = np.frombuffer(buf, dtype=np.float64).reshape(7, b + 1).copy()
    return tab, (int(m[0]), float(m[1]), float(m[2]), int(m[3]))


@dataclass(frozen=True)
class Cosmology:
    """Background (guide Ch. 5: H0, Omega_m, Omega_Lambda); H0 in the inverse
    time unit of the simulation."""
    H0: float
    Omega_m: float
    Omega_L: float = 0.0

    def _c(self):
        return P3MCosmology(float(self.H0), float(self.Omega_m), float(self.Omega_L))

    def age(self, a: float) -> float:
        out = ctypes.c_double()
        _check(_lib.p3m_cosmo_age(ctypes.byref(self._c()), float(a), ctypes.byref(out)),
               "p3m_cosmo_age")
        return out.value

    def scale_factor(self, t: float) -> float:
        out = ctypes.c_double()
        _check(_lib.p3m_cosmo_scale_factor(ctypes.byref(self._c()), float(t),
                                           ctypes.byref(out)), "p3m_cosmo_scale_factor")
        return out.value

    def kick_drift(self, a0: float, a1: float):
        """(c_kick, c_drift) = (int dt/a, int dt/a^2) from a0 to a1."""
        ck, cd = ctypes.c_double(), ctypes.c_double()
        _check(_lib.p3m_cosmo_kick_drift(ctypes.byref(self._c()), float(a0), float(a1),
                                         ctypes.byref(ck), ctypes.byref(cd)),
               "p3m_cosmo_kick_drift")
        return ck.value, cd.value

    def kdk_step(self, a: float, dt_factor: float):
        """One kick-drift-kick step of length dt_factor times the age at a
        (guide Ch. 5, Delta t_factor): returns (a_next, c_kick_first, c_drift,
        c_kick_second), the kicks covering the first and second half in time
        (p3m_cosmo_kdk_step)."""
        out = [ctypes.c_double() for _ in range(4)]
        _check(_lib.p3m_cosmo_kdk_step(ctypes.byref(self._c()), float(a), float(dt_factor),
                                       *[ctypes.byref(o) for o in out]), "p3m_cosmo_kdk_step")
        return tuple(o.value for o in out)


@dataclass
class Params:
    """Plan parameters (guide Ch. 5: PM_gridsize, boxsize, PM_scale,
    P3M_cutoff, softeningfactors; the softening here is an absolute length)."""
    grid_n: int
    box: float = 1.0
    rs_cells: float = 1.25
    cutoff_rs: float = 4.5
    softening: float = 0.0
    G: float = 1.0
    precision: str = "fp32"      # "fp32" or "fp64"
    fd_order: int = 4
    deconv_power: int = 2
    adjoint: bool = False        # also allocate the workspace of the VJP calls
    ewald_gridsize: int = 0      # > 0: tabulate the Ewald correction (pp_ewald_force)
    pair_partials: int = 0       # < 0: every pair from both sides; else partials per
                                 # particle of the one-sided sum (0: the default)

    def to_c(self) -> P3MParams:
        if self.precision not in ("fp32", "fp64"):
            raise ValueError("precision must be 'fp32' or 'fp64'")
        return P3MParams(int(self.grid_n),
                         P3M_FP32 if self.precision == "fp32" else P3M_FP64,
                         int(self.fd_order), int(self.deconv_power), float(self.box),
                         float(self.rs_cells), float(self.cutoff_rs),
                         float(self.softening), float(self.G), 1 if self.adjoint else 0,
                         int(self.ewald_gridsize), int(self.pair_partials))


def pp_force_noalloc(params: Params, pos, mass=None, out=None, fp32_out=False):
    """pp_force without a plan (the library's fixed workspace; no device
    allocation inside the call): short-range force, shape (3, n)."""
    n = _vec3(pos, "pos")
    m, ms = _mass(mass, n)
    if out is None:
        out = torch.empty((3, n), dtype=torch.float32 if fp32_out else torch.float64,
                          device=pos.device)
    else:
        fp32_out = out.dtype == torch.float32
        if _vec3(out, "out", out.dtype) != n or out.dtype not in (torch.float32, torch.float64):
            raise ValueError("out must be (3, n) float32 or float64")
    c = params.to_c()
    _check(_lib.pp_force_noalloc(ctypes.byref(c), n, _ptr(pos), _ptr(m), ms, _ptr(out),
                                 1 if fp32_out else 0, _stream_ptr()), "pp_force_noalloc")
    return out


class Plan:
    """Owns a libp3m plan (workspace for up to ``n_max`` particles)."""

    def __init__(self, params: Params, n_max: int, stream=None):
        self.params = params
        self.n_max = int(n_max)
        c = params.to_c()
        h = ctypes.c_void_p()
        _check(_lib.p3m_plan_create(ctypes.byref(c), self.n_max, _stream_ptr(stream),
                                    ctypes.byref(h)), "p3m_plan_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(_lib.p3m_plan_destroy(self._h), "p3m_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _handle(self):
        if self._h is None:
            raise ValueError("plan is closed")
        _check(_lib.p3m_plan_set_stream(self._h, _stream_ptr()), "p3m_plan_set_stream")
        return self._h

    def _force(self, fn, name, pos, mass, out, fp32_out):
        n = _vec3(pos, "pos")
        m, ms = _mass(mass, n)
        if out is None:
            out = torch.empty((3, n), dtype=torch.float32 if fp32_out else torch.float64,
                              device=pos.device)
        else:
            fp32_out = out.dtype == torch.float32
            if _vec3(out, "out", out.dtype) != n or out.dtype not in (torch.float32,
                                                                      torch.float64):
                raise ValueError("out must be (3, n) float32 or float64")
        _check(fn(self._handle(), n, _ptr(pos), _ptr(m), ms, _ptr(out),
                  1 if fp32_out else 0), name)
        return out

    def force(self, pos, mass=None, out=None, fp32_out=False):
        """Full P3M force F = m (a_PP + a_PM), shape (3, n)."""
        return self._force(_lib.p3m_force, "p3m_force", pos, mass, out, fp32_out)

    def force_cell_order(self, pos, mass=None, out=None, order=None, fp32_out=False):
        """The P3M force in the cell order of this call's binning: returns
        (F, order) with F[:, s] the force on input particle order[s]."""
        n = _vec3(pos, "pos")
        if order is None:
            order = torch.empty(n, dtype=torch.int32, device=pos.device)
        elif order.dtype != torch.int32 or order.shape != (n,) or not order.is_contiguous():
            raise ValueError("order must be a contiguous int32 tensor of n entries")

        def fn(h, n_, p, m, ms, f, f32):
            return _lib.p3m_force_cell_order(h, n_, p, m, ms, f, f32, _ptr(order))
        return self._force(fn, "p3m_force_cell_order", pos, mass, out, fp32_out), order

    def pm_force(self, pos, mass=None, out=None, fp32_out=False):
        return self._force(_lib.pm_force, "pm_force", pos, mass, out, fp32_out)

    def pp_force(self, pos, mass=None, out=None, fp32_out=False):
        return self._force(_lib.pp_force, "pp_force", pos, mass, out, fp32_out)

    def _vjp(self, fn, name, pos, mass, force_bar, out):
        n = _vec3(pos, "pos")
        if _vec3(force_bar, "force_bar") != n:
            raise ValueError("force_bar must match pos")
        m, ms = _mass(mass, n)
        if out is None:
            out = torch.empty((3, n), dtype=torch.float64, device=pos.device)
        elif _vec3(out, "out") != n:
            raise ValueError("out must be a (3, n) float64 tensor")
        _check(fn(self._handle(), n, _ptr(pos), _ptr(m), ms, _ptr(force_bar), _ptr(out)), name)
        return out

    def force_vjp(self, pos, mass, force_bar, out=None):
        """pos_bar = force_bar . dF/dpos of the full P3M force (plan made with
        Params(adjoint=True)), shape (3, n) float64."""
        return self._vjp(_lib.p3m_force_vjp, "p3m_force_vjp", pos, mass, force_bar, out)

    def pm_force_vjp(self, pos, mass, force_bar, out=None):
        return self._vjp(_lib.pm_force_vjp, "pm_force_vjp", pos, mass, force_bar, out)

    def pp_force_vjp(self, pos, mass, force_bar, out=None):
        return self._vjp(_lib.pp_force_vjp, "pp_force_vjp", pos, mass, force_bar, out)

    def pp_ewald_force(self, pos, mass=None, out=None, fp32_out=False):
        """All-pairs PP force with the tabulated Ewald correction (plan made
        with Params(ewald_gridsize=E)), shape (3, n)."""
        return self._force(_lib.pp_ewald_force, "pp_ewald_force", pos, mass, out, fp32_out)

    def ewald_correction(self, r):
        """Tabulated correction c(r) at separations r ((3, npts) float64)."""
        npts = _vec3(r, "r")
        out = torch.empty_like(r)
        _check(_lib.p3m_ewald_correction(self._handle(), npts, _ptr(r), _ptr(out)),
               "p3m_ewald_correction")
        return out

    def power_spectrum(self, pos, mass=None, nbins=None, r_tophat=0.0):
        """(k, P, modes, sigma) of the particle density on the plan's grid:
        shell-mean |k|, shell-mean power and mode count per unit-width shell
        in |n| (nbins, default grid_n / 2), and sigma(r_tophat); device float64."""
        n = _vec3(pos, "pos")
        m, ms = _mass(mass, n)
        nb = int(nbins if nbins is not None else self.params.grid_n // 2)
        out = torch.empty((3, max(nb, 1)), dtype=torch.float64, device=pos.device)
        sig = torch.empty(1, dtype=torch.float64, device=pos.device)
        _check(_lib.p3m_power_spectrum(self._handle(), n, _ptr(pos), _ptr(m), ms, nb,
                                       float(r_tophat), _ptr(out[0]), _ptr(out[1]),
                                       _ptr(out[2]), _ptr(sig)), "p3m_power_spectrum")
        return out[0], out[1], out[2], sig[0]

    def pair_count(self, pos) -> int:
        """Ordered pairs with 0 < r < r_c (synchronises to return the count)."""
        n = _vec3(pos, "pos")
        cnt = torch.zeros(1, dtype=torch.int64, device=pos.device)
        _check(_lib.p3m_pair_count(self._handle(), n, _ptr(pos), _ptr(cnt)),
               "p3m_pair_count")
        return int(cnt.item())

    def set_timing(self, capacity: int):
        """Record stage events for the next ``capacity`` force calls (0: off)."""
        _check(_lib.p3m_set_timing(self._handle(), int(capacity)), "p3m_set_timing")

    def stage_times(self):
        """(calls recorded, {stage: total ms over those calls}); synchronises."""
        buf = (ctypes.c_double * len(STAGES))()
        n = _lib.p3m_stage_times(self._h, buf, len(STAGES))
        _check(min(n, 0), "p3m_stage_times")
        return n, {k: float(v) for k, v in zip(STAGES, buf)}


def kick(mom: torch.Tensor, force: torch.Tensor, c_kick: float) -> torch.Tensor:
    """p <- p + c_kick F in place (FP64 momenta; F float32 or float64)."""
    n = _vec3(mom, "mom")
    if _vec3(force, "force", force.dtype) != n or force.dtype not in (torch.float32,
                                                                       torch.float64):
        raise ValueError("force must be (3, n) float32 or float64")
    _check(_lib.p3m_kick(n, _ptr(mom), _ptr(force), 1 if force.dtype == torch.float32 else 0,
                         float(c_kick), _stream_ptr()), "p3m_kick")
    return mom


def kick_reorder(order: torch.Tensor, pos: torch.Tensor, mom: torch.Tensor,
                 force: torch.Tensor, c_kick: float, ids=None, mass=None, out=None):
    """Second half-kick of a step in cell order: with i = order[s],
    mom_out[:, s] = mom[:, i] + c_kick force[:, s] and pos_out[:, s] =
    pos[:, i] (ids and a per-particle mass array carried along). `force` is
    in cell order (Plan.force_cell_order). Returns (pos_out, mom_out,
    ids_out, mass_out); `out` may give those buffers (None entries are
    allocated)."""
    n = _vec3(pos, "pos")
    if mass is not None and not isinstance(mass, torch.Tensor):
        mass = None                      # a scalar mass needs no reordering
    if _vec3(mom, "mom") != n:
        raise ValueError("mom must match pos")
    if _vec3(force, "force", force.dtype) != n or force.dtype not in (torch.float32,
                                                                       torch.float64):
        raise ValueError("force must be (3, n) float32 or float64")
    if order.dtype != torch.int32 or order.shape != (n,) or not order.is_contiguous():
        raise ValueError("order must be a contiguous int32 tensor of n entries")
    for name, t, dt in (("ids", ids, torch.int64), ("mass", mass, torch.float64)):
        if t is not None and (t.dtype != dt or t.shape != (n,) or not t.is_contiguous()
                              or t.device != pos.device):
            raise ValueError(f"{name} must be a contiguous {dt} device tensor of n entries")
    po, mo, io, ma = out if out is not None else (None, None, None, None)
    po = torch.empty_like(pos) if po is None else po
    mo = torch.empty_like(mom) if mo is None else mo
    if ids is not None and io is None:
        io = torch.empty_like(ids)
    if mass is not None and ma is None:
        ma = torch.empty_like(mass)
    if _vec3(po, "pos_out") != n or _vec3(mo, "mom_out") != n:
        raise ValueError("pos_out and mom_out must be (3, n) float64")
    _check(_lib.p3m_kick_reorder(n, _ptr(order), _ptr(pos), _ptr(mom), _ptr(force),
                                 1 if force.dtype == torch.float32 else 0, _ptr(ids), _ptr(mass),
                                 float(c_kick), _ptr(po), _ptr(mo),
                                 _ptr(io) if ids is not None else None,
                                 _ptr(ma) if mass is not None else None, _stream_ptr()),
           "p3m_kick_reorder")
    return po, mo, io, ma


def kick_drift(pos: torch.Tensor, mom: torch.Tensor, force: torch.Tensor, mass,
               c_kick: float, c_drift: float, box: float):
    """p <- p + c_kick F, then x <- wrap(x + c_drift p / m), in place, in one
    pass (bitwise the same as kick followed by drift)."""
    n = _vec3(pos, "pos")
    if _vec3(mom, "mom") != n:
        raise ValueError("mom must match pos")
    if _vec3(force, "force", force.dtype) != n or force.dtype not in (torch.float32,
                                                                       torch.float64):
        raise ValueError("force must be (3, n) float32 or float64")
    m, ms = _mass(mass, n)
    _check(_lib.p3m_kick_drift(n, _ptr(pos), _ptr(mom), _ptr(force),
                               1 if force.dtype == torch.float32 else 0, _ptr(m), ms,
                               float(c_kick), float(c_drift), float(box), _stream_ptr()),
           "p3m_kick_drift")
    return pos, mom


def drift_vjp(mom_bar: torch.Tensor, pos_bar: torch.Tensor, mass, c_drift: float):
    """Transpose of the drift: p_bar <- p_bar + (c_drift / m) x_bar in place."""
    n = _vec3(mom_bar, "mom_bar")
    if _vec3(pos_bar, "pos_bar") != n:
        raise ValueError("pos_bar must match mom_bar")
    m, ms = _mass(mass, n)
    _check(_lib.p3m_drift_vjp(n, _ptr(mom_bar), _ptr(pos_bar), _ptr(m), ms, float(c_drift),
                              _stream_ptr()), "p3m_drift_vjp")
    return mom_bar


def drift(pos: torch.Tensor, mom: torch.Tensor, mass, c_drift: float, box: float):
    """x <- wrap(x + c_drift p / m) in place."""
    n = _vec3(pos, "pos")
    if _vec3(mom, "mom") != n:
        raise ValueError("mom must match pos")
    m, ms = _mass(mass, n)
    _check(_lib.p3m_drift(n, _ptr(pos), _ptr(mom), _ptr(m), ms, float(c_drift), float(box),
                          _stream_ptr()), "p3m_drift")
    return pos
