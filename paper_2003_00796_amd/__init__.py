"""Python binding of libmcx: MI355X (gfx950) Monte-Carlo electron-photon dose
transport behind a C ABI (include/mcx.h).

The binding only marshals arguments (ctypes); every step of the particle-
history loop runs in the library's HIP kernels.  PyTorch supplies device
memory and streams where a caller passes tensors.  If the compiled library is
missing, importing works but creating a Simulator raises: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmcx.so")

FP64, MIXED = 0, 1
PHOTON, ELECTRON, POSITRON = 0, 1, 2
SRC_PENCIL, SRC_RECT = 0, 1
NO_COMPTON, NO_PHOTO, NO_RAYLEIGH, NO_PAIR = 1, 2, 4, 8
NO_HARD_ELASTIC, NO_HARD_INELASTIC, NO_HARD_BREMS = 16, 32, 64
STRAGGLING = 128
ANNIH_FLIGHT = 256
# mcx_set_gradient: score the soft deflection's energy dependence (term E)
GRAD_DEFLECTION_ENERGY = 1

ERRORS = {0: "MCX_OK", -1: "MCX_E_INVALID", -2: "MCX_E_STATE", -3: "MCX_E_NOMEM", -4: "MCX_E_DEVICE",
          -5: "MCX_E_RANGE", -6: "MCX_E_CANCELLED", -7: "MCX_E_UNSUPPORTED"}

# every symbol the C ABI exports (include/mcx.h)
ABI_SYMBOLS = ("mcx_create", "mcx_destroy", "mcx_last_error", "mcx_set_transport", "mcx_load_material",
               "mcx_load_phantom", "mcx_set_sources", "mcx_set_launch", "mcx_set_timing", "mcx_set_test_mode", "mcx_run",
               "mcx_get_dose", "mcx_get_tally", "mcx_reset_tallies", "mcx_get_stats",
               "mcx_get_history_results", "mcx_dose_backward", "mcx_set_graph", "mcx_autotune",
               "mcx_synchronize", "mcx_cancel", "mcx_checkpoint", "mcx_restore", "mcx_workspace_size",
               "mcx_set_workspace", "mcx_set_influence", "mcx_get_influence", "mcx_ct_to_phantom",
               "mcx_run_static", "mcx_set_gradient")


class MaterialDesc(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "z_mol", "a_mol", "zz1_mol", "z_screen", "i_exc", "pe_coef", "pe_eref", "pe_exp", "pp_coef",
        "ray_f0", "ray_a", "brems_b")]


class Transport(C.Structure):
    _fields_ = [("n_grid", C.c_int), ("e_min", C.c_double), ("e_max", C.c_double),
                ("eabs", C.c_double * 3), ("c1", C.c_double), ("c2", C.c_double),
                ("wcc", C.c_double), ("wcr", C.c_double), ("flags", C.c_uint32),
                ("force_in", C.c_double), ("force_br", C.c_double), ("split_br", C.c_int)]


class PhantomDesc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("voxel_cm", C.c_double * 3),
                ("origin_cm", C.c_double * 3), ("rho", C.c_void_p), ("rho_on_device", C.c_int),
                ("mat", C.c_void_p)]


class Source(C.Structure):
    _fields_ = [("particle", C.c_int), ("kind", C.c_int), ("energy", C.c_double),
                ("pos", C.c_double * 3), ("dir", C.c_double * 3), ("width", C.c_double * 2),
                ("n_hist", C.c_uint64)]


class CTCalibration(C.Structure):
    _fields_ = [("n_points", C.c_int), ("hu", C.c_void_p), ("rho", C.c_void_p), ("n_thresholds", C.c_int),
                ("mat_hu", C.c_void_p)]


def ct_to_phantom(hu, hu_points, rho_points, mat_thresholds=()):
    """(rho, mat) arrays of the shape of `hu` from a CT calibration:
    piecewise-linear HU -> density through (hu_points, rho_points), and the
    material index = number of thresholds at or below each HU (host code,
    mcx_ct_to_phantom)."""
    h = np.ascontiguousarray(hu, dtype=np.int16)
    xp = np.ascontiguousarray(hu_points, dtype=np.float64)
    fp = np.ascontiguousarray(rho_points, dtype=np.float64)
    th = np.ascontiguousarray(mat_thresholds, dtype=np.float64)
    cal = CTCalibration(n_points=len(xp), hu=xp.ctypes.data, rho=fp.ctypes.data, n_thresholds=len(th),
                        mat_hu=th.ctypes.data if len(th) else None)
    rho = np.zeros(h.shape)
    mat = np.zeros(h.shape, dtype=np.uint8)
    rc = lib().mcx_ct_to_phantom(C.byref(cal), h.ctypes.data, h.size, rho.ctypes.data, mat.ctypes.data)
    if rc != 0:
        raise MCXError(f"mcx_ct_to_phantom: {ERRORS.get(rc, rc)}")
    return rho, mat


_STATS_U64_A = ("histories", "flights", "compton", "photo", "rayleigh", "pair", "esteps", "hard_el", "hard_in",
                "hard_br", "delta", "annih", "crossings", "secondaries", "deposits", "absorbed", "escaped")


class Stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in _STATS_U64_A] + [
        ("e_dep", C.c_double), ("e_esc", C.c_double), ("pos_esc", C.c_uint64), ("iterations", C.c_uint64),
        ("chunks", C.c_uint64), ("tally_pairs", C.c_uint64), ("ms_transport", C.c_double),
        ("ms_flush", C.c_double), ("evisits", C.c_uint64), ("ewrites", C.c_uint64), ("inserts", C.c_uint64),
        ("ms_source", C.c_double), ("ms_flight", C.c_double), ("ms_knock", C.c_double), ("ms_estep", C.c_double),
        ("timed_iterations", C.c_uint64), ("ms_backward", C.c_double), ("next_history", C.c_uint64),
        ("annih_flight", C.c_uint64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class MCXError(RuntimeError):
    pass


class MCXCancelled(MCXError):
    """mcx_run honoured mcx_cancel: histories [first, next_history) are
    complete and in the tallies."""

    def __init__(self, msg: str, next_history: int):
        super().__init__(msg)
        self.next_history = next_history


_lib = None


def lib():
    """Load libmcx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # One HIP runtime per process: PyTorch ships its own libamdhip64 with
        # the same soname, so load it first and libmcx binds to that copy
        # (loading the system runtime first leaves PyTorch without a device).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise MCXError(f"{LIB_PATH} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.mcx_create.argtypes = [C.POINTER(vp), C.c_int, C.c_int]
        L.mcx_destroy.argtypes = [vp]
        L.mcx_destroy.restype = None
        L.mcx_last_error.argtypes = [vp]
        L.mcx_last_error.restype = C.c_char_p
        L.mcx_set_transport.argtypes = [vp, C.POINTER(Transport)]
        L.mcx_load_material.argtypes = [vp, C.c_int, C.POINTER(MaterialDesc)]
        L.mcx_load_phantom.argtypes = [vp, C.POINTER(PhantomDesc)]
        L.mcx_set_sources.argtypes = [vp, C.POINTER(Source), C.c_int]
        L.mcx_set_launch.argtypes = [vp, C.c_uint32, C.c_uint32, C.c_uint32]
        L.mcx_set_test_mode.argtypes = [vp, C.c_int]
        L.mcx_set_timing.argtypes = [vp, C.c_int]
        L.mcx_set_gradient.argtypes = [vp, C.c_uint32]
        L.mcx_run.argtypes = [vp, C.c_uint64, C.c_uint64, C.c_uint64, vp]
        L.mcx_run_static.argtypes = [vp, C.c_uint64, C.c_uint64, C.c_uint64, vp]
        L.mcx_get_dose.argtypes = [vp, vp, vp, C.c_int, vp]
        L.mcx_get_tally.argtypes = [vp, vp, vp, C.c_int, vp]
        L.mcx_reset_tallies.argtypes = [vp]
        L.mcx_get_stats.argtypes = [vp, C.POINTER(Stats)]
        L.mcx_get_history_results.argtypes = [vp, vp, vp]
        L.mcx_dose_backward.argtypes = [vp, vp, vp, C.c_int, vp]
        L.mcx_set_graph.argtypes = [vp, C.c_int]
        L.mcx_autotune.argtypes = [vp, C.c_uint64, C.c_char_p, C.POINTER(C.c_uint32)]
        L.mcx_synchronize.argtypes = [vp]
        L.mcx_cancel.argtypes = [vp]
        L.mcx_checkpoint.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
        L.mcx_restore.argtypes = [vp, vp, C.c_size_t]
        L.mcx_workspace_size.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.mcx_set_workspace.argtypes = [vp, vp, C.c_size_t]
        L.mcx_set_influence.argtypes = [vp, C.c_int, C.c_uint32]
        L.mcx_ct_to_phantom.argtypes = [C.POINTER(CTCalibration), vp, C.c_uint64, vp, vp]
        L.mcx_get_influence.argtypes = [vp, vp, vp, vp, vp, C.c_uint64, C.POINTER(C.c_uint64)]
        for f in ABI_SYMBOLS:
            if f not in ("mcx_destroy", "mcx_last_error"):
                getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return C.c_void_p(a.ctypes.data)


class Simulator:
    """One library context: material, phantom, sources, tallies.

    material: dict of MaterialDesc fields; transport: dict with n_grid, e_min,
    e_max, eabs (3), c1, c2, wcc, wcr, flags; phantom: dict with shape
    (nz, ny, nx), voxel (dx, dy, dz), origin, rho (numpy array or torch
    tensor, float64); sources: list of dicts (particle, kind, energy, pos, dir,
    width, n_hist).
    """

    def __init__(self, precision: int = FP64, device: int = 0):
        self._L = lib()
        self._h = C.c_void_p()
        rc = self._L.mcx_create(C.byref(self._h), device, precision)
        if rc != 0:
            raise MCXError(f"mcx_create failed: {ERRORS.get(rc, rc)}")
        self.precision = precision
        self.shape = None
        self.n_hist_total = 0
        self._workspace = None  # device tensor the context carves its run memory from

    def close(self):
        if self._h:
            self._L.mcx_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, what: str):
        if rc != 0:
            msg = self._L.mcx_last_error(self._h).decode(errors="replace")
            raise MCXError(f"{what}: {ERRORS.get(rc, rc)}: {msg}")

    def set_transport(self, t: dict):
        s = Transport()
        s.n_grid = int(t["n_grid"])
        s.e_min, s.e_max = float(t["e_min"]), float(t["e_max"])
        for i in range(3):
            s.eabs[i] = float(t["eabs"][i])
        s.c1, s.c2, s.wcc, s.wcr = (float(t[k]) for k in ("c1", "c2", "wcc", "wcr"))
        s.flags = int(t.get("flags", 0))
        s.force_in = float(t.get("force_in", 0.0))
        s.force_br = float(t.get("force_br", 0.0))
        s.split_br = int(t.get("split_br", 0))
        self._check(self._L.mcx_set_transport(self._h, C.byref(s)), "set_transport")

    def load_material(self, m: dict, mat_id: int = 0):
        d = MaterialDesc(**{k: float(m[k]) for k, _ in MaterialDesc._fields_})
        self._check(self._L.mcx_load_material(self._h, mat_id, C.byref(d)), "load_material")

    def load_phantom(self, ph: dict):
        nz, ny, nx = ph["shape"]
        rho = ph["rho"]
        d = PhantomDesc(nx=nx, ny=ny, nz=nz)
        for k in range(3):
            d.voxel_cm[k] = float(ph["voxel"][k])
            d.origin_cm[k] = float(ph["origin"][k])
        keep = None
        if hasattr(rho, "data_ptr") and getattr(rho, "is_cuda", False):
            keep = rho.contiguous().double()
            d.rho = C.c_void_p(keep.data_ptr())
            d.rho_on_device = 1
        else:
            keep = np.ascontiguousarray(np.asarray(rho, dtype=np.float64))
            d.rho = C.c_void_p(keep.ctypes.data)
            d.rho_on_device = 0
        mat = ph.get("mat")
        if mat is not None:
            mkeep = np.ascontiguousarray(np.asarray(mat, dtype=np.uint8))
            assert mkeep.size == nx * ny * nz
            d.mat = C.c_void_p(mkeep.ctypes.data)
        self._check(self._L.mcx_load_phantom(self._h, C.byref(d)), "load_phantom")
        self.shape = (nz, ny, nx)

    def set_sources(self, sources):
        arr = (Source * len(sources))()
        for i, s in enumerate(sources):
            arr[i].particle = int(s["particle"])
            arr[i].kind = int(s["kind"])
            arr[i].energy = float(s["energy"])
            for k in range(3):
                arr[i].pos[k] = float(s["pos"][k])
                arr[i].dir[k] = float(s["dir"][k])
            w = s.get("width", (0.0, 0.0))
            arr[i].width[0], arr[i].width[1] = float(w[0]), float(w[1])
            arr[i].n_hist = int(s["n_hist"])
        self._check(self._L.mcx_set_sources(self._h, arr, len(sources)), "set_sources")
        self.n_hist_total = sum(int(s["n_hist"]) for s in sources)

    def set_launch(self, bank: int = 0, block: int = 0, steps: int = 0):
        self._check(self._L.mcx_set_launch(self._h, bank, block, steps), "set_launch")

    def set_gradient(self, flags: int):
        """Options of the density gradient (GRAD_DEFLECTION_ENERGY)."""
        self._check(self._L.mcx_set_gradient(self._h, int(flags)), "set_gradient")
        return self

    def set_timing(self, on: bool):
        self._check(self._L.mcx_set_timing(self._h, 1 if on else 0), "set_timing")

    def set_graph(self, on: bool):
        self._check(self._L.mcx_set_graph(self._h, 1 if on else 0), "set_graph")

    def autotune(self, n_sample: int = 0, cache_path: str | None = None):
        """(bank, block, steps) chosen by timing a sample; see mcx_autotune."""
        out = (C.c_uint32 * 3)()
        self._check(self._L.mcx_autotune(self._h, n_sample, cache_path.encode() if cache_path else None, out),
                    "autotune")
        return tuple(out)

    def set_test_mode(self, on: bool):
        self._check(self._L.mcx_set_test_mode(self._h, 1 if on else 0), "set_test_mode")

    def setup(self, workload: dict):
        """material + transport + phantom + sources from a workload dict."""
        self.set_transport(workload["transport"])
        for k, m in enumerate(workload.get("materials") or [workload["material"]]):
            self.load_material(m, k)
        self.load_phantom(workload["phantom"])
        self.set_sources(workload["sources"])
        return self

    def run(self, seed: int, first: int, n: int, stream=None):
        """Histories [first, first + n); raises MCXCancelled (with the
        watermark) when the run honoured a cancel request."""
        sp = C.c_void_p(stream) if stream else None
        rc = self._L.mcx_run(self._h, seed, first, n, sp)
        if rc == -6:
            msg = self._L.mcx_last_error(self._h).decode(errors="replace")
            raise MCXCancelled(f"run: MCX_E_CANCELLED: {msg}", self.stats()["next_history"])
        self._check(rc, "run")

    def run_static(self, seed: int, first: int, n: int, stream=None):
        """Histories [first, first + n) in the library's fixed device array
        (mcx_run_static: the call allocates nothing)."""
        sp = C.c_void_p(stream) if stream else None
        rc = self._L.mcx_run_static(self._h, seed, first, n, sp)
        if rc == -6:
            msg = self._L.mcx_last_error(self._h).decode(errors="replace")
            raise MCXCancelled(f"run_static: MCX_E_CANCELLED: {msg}", self.stats()["next_history"])
        self._check(rc, "run_static")

    def cancel(self):
        """Ask the run in progress (or the next one) to stop; thread-safe."""
        self._check(self._L.mcx_cancel(self._h), "cancel")

    def synchronize(self):
        self._check(self._L.mcx_synchronize(self._h), "synchronize")

    def checkpoint(self) -> bytes:
        n = C.c_size_t(0)
        self._check(self._L.mcx_checkpoint(self._h, None, C.byref(n)), "checkpoint")
        buf = C.create_string_buffer(n.value)
        self._check(self._L.mcx_checkpoint(self._h, buf, C.byref(n)), "checkpoint")
        return buf.raw[:n.value]

    def restore(self, data: bytes):
        buf = C.create_string_buffer(bytes(data), len(data))
        self._check(self._L.mcx_restore(self._h, buf, len(data)), "restore")

    def set_influence(self, on: bool = True, log2_slots: int = 24):
        """Per-source (beamlet) dose influence: (source, voxel) Sum q and
        Sum q^2 accumulated by later runs (see mcx_set_influence)."""
        self._check(self._L.mcx_set_influence(self._h, 1 if on else 0, log2_slots), "set_influence")

    def influence_count(self) -> int:
        """Number of (source, voxel) entries in the influence table."""
        n = C.c_uint64(0)
        self._check(self._L.mcx_get_influence(self._h, None, None, None, None, 0, C.byref(n)), "get_influence")
        return n.value

    def influence(self, sort: bool = True):
        """(source, voxel, sum_q, sum_q2) arrays of the influence table,
        sorted by source, then voxel (sort=False: in the library's order,
        which saves a host sort of every entry)."""
        k = self.influence_count()
        src = np.zeros(k, dtype=np.uint32)
        vox = np.zeros(k, dtype=np.uint32)
        q = np.zeros(k)
        q2 = np.zeros(k)
        if k:
            n = C.c_uint64(0)
            self._check(self._L.mcx_get_influence(self._h, _ptr(src), _ptr(vox), _ptr(q), _ptr(q2), k, C.byref(n)),
                        "get_influence")
            if n.value != k:
                raise RuntimeError(f"influence table changed between the count ({k}) and the read ({n.value})")
        if not sort:
            return src, vox, q, q2
        order = np.lexsort((vox, src))
        return src[order], vox[order], q[order], q2[order]

    def workspace_size(self) -> int:
        n = C.c_size_t(0)
        self._check(self._L.mcx_workspace_size(self._h, C.byref(n)), "workspace_size")
        return n.value

    def set_workspace(self, buf=None):
        """Carve the run's queues, counters and tally table from a device
        tensor (kept referenced here); None returns to library memory."""
        if buf is None:
            self._check(self._L.mcx_set_workspace(self._h, None, 0), "set_workspace")
            self._workspace = None
            return
        self._check(self._L.mcx_set_workspace(self._h, C.c_void_p(buf.data_ptr()),
                                              buf.numel() * buf.element_size()), "set_workspace")
        self._workspace = buf

    def reset(self):
        self._check(self._L.mcx_reset_tallies(self._h), "reset_tallies")

    def dose(self):
        """(dose, sigma) in eV/g per history as numpy arrays of the phantom shape."""
        nv = int(np.prod(self.shape))
        d = np.zeros(nv)
        s = np.zeros(nv)
        self._check(self._L.mcx_get_dose(self._h, _ptr(d), _ptr(s), 0, None), "get_dose")
        return d.reshape(self.shape), s.reshape(self.shape)

    def dose_into(self, dose_t, sigma_t=None, stream=None):
        """Write dose (and sigma) into device tensors (float64, contiguous)."""
        sp = C.c_void_p(stream) if stream else None
        self._check(self._L.mcx_get_dose(self._h, C.c_void_p(dose_t.data_ptr()),
                                          C.c_void_p(sigma_t.data_ptr()) if sigma_t is not None else None, 1, sp),
                    "get_dose")

    def tally(self):
        nv = int(np.prod(self.shape))
        q = np.zeros(nv)
        q2 = np.zeros(nv)
        self._check(self._L.mcx_get_tally(self._h, _ptr(q), _ptr(q2), 0, None), "get_tally")
        return q, q2

    def stats(self) -> dict:
        s = Stats()
        self._check(self._L.mcx_get_stats(self._h, C.byref(s)), "get_stats")
        return s.as_dict()

    def dose_backward(self, dl_ddose: np.ndarray) -> np.ndarray:
        """dL/drho for dL/dD = dl_ddose (host arrays of the phantom shape)."""
        g = np.ascontiguousarray(dl_ddose, dtype=np.float64)
        out = np.zeros_like(g)
        self._check(self._L.mcx_dose_backward(self._h, _ptr(g), _ptr(out), 0, None), "dose_backward")
        return out

    def dose_backward_into(self, dl_ddose_t, out_t, stream=None):
        """Device variant: float64 contiguous tensors."""
        sp = C.c_void_p(stream) if stream else None
        self._check(self._L.mcx_dose_backward(self._h, C.c_void_p(dl_ddose_t.data_ptr()),
                                               C.c_void_p(out_t.data_ptr()), 1, sp), "dose_backward")

    def history_results(self, n: int):
        h = np.zeros(n, dtype=np.uint64)
        led = np.zeros((n, 3))
        self._check(self._L.mcx_get_history_results(self._h, _ptr(h), _ptr(led)), "get_history_results")
        return h, led


class DoseModel:
    """A fixed transport problem whose voxel densities are the input: the dose
    it produces is differentiable through DoseFunction."""

    def __init__(self, workload: dict, n_hist: int, seed: int = 1, precision: int = FP64, device: int = 0):
        self.sim = Simulator(precision, device)
        self.sim.set_transport(workload["transport"])
        self.sim.load_material(workload["material"])
        self.workload = workload
        self.n_hist = int(n_hist)
        self.seed = int(seed)
        self._sources_set = False

    def forward(self, rho):
        import torch
        ph = dict(self.workload["phantom"], rho=rho.detach())
        self.sim.load_phantom(ph)
        if not self._sources_set:
            self.sim.set_sources(self.workload["sources"])
            self._sources_set = True
        stream = torch.cuda.current_stream(rho.device).cuda_stream
        self.sim.run(self.seed, 0, self.n_hist, stream)
        dose = torch.empty(self.sim.shape, dtype=torch.float64, device=rho.device)
        self.dose_sigma = torch.empty_like(dose)
        self.sim.dose_into(dose, self.dose_sigma, stream)
        return dose

    def backward(self, grad_dose):
        import torch
        g = grad_dose.contiguous().double()
        out = torch.empty_like(g)
        self.sim.dose_backward_into(g, out, torch.cuda.current_stream(g.device).cuda_stream)
        return out


def _dose_function():
    import torch

    class DoseFunction(torch.autograd.Function):
        """dose = DoseFunction.apply(rho, model): Monte-Carlo dose (eV/g per
        history) of `model` with voxel densities rho (float64 CUDA tensor of
        the phantom shape); backward replays the histories on the GPU."""

        @staticmethod
        def forward(ctx, rho, model):
            ctx.model = model
            return model.forward(rho)

        @staticmethod
        def backward(ctx, grad_dose):
            return ctx.model.backward(grad_dose), None

    return DoseFunction


_DOSE_FUNCTION = None


def __getattr__(name):
    global _DOSE_FUNCTION
    if name == "DoseFunction":
        if _DOSE_FUNCTION is None:
            _DOSE_FUNCTION = _dose_function()
        return _DOSE_FUNCTION
    raise AttributeError(name)
