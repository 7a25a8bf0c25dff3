"""ctypes binding of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and by
the CPU-baseline leg of the benchmark.  The product package never imports it.
The oracle is a plain single-thread reference transport of the paper's
independent particle-history loop (arXiv:2003.00796, Sec. 4.1 JUMP/STEP/KNOCK,
Sec. 4.3 Eq. (1)-(3) estimators); see oracle.h for the readings.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

PHOTON, ELECTRON, POSITRON = 0, 1, 2
SRC_PENCIL, SRC_RECT = 0, 1

NO_COMPTON, NO_PHOTO, NO_RAYLEIGH, NO_PAIR = 1, 2, 4, 8
NO_HARD_ELASTIC, NO_HARD_INELASTIC, NO_HARD_BREMS = 16, 32, 64
STRAGGLING = 128
ANNIH_FLIGHT = 256
GRAD_DEFLECTION_ENERGY = 512

# orc_eval channels
MU_COMPTON, MU_PHOTO, MU_RAYLEIGH, MU_PAIR = 0, 1, 2, 3


def ech(ptype: int, c: int) -> int:
    """Electron (ptype 0) / positron (1) table channel c: 0 S_soft, 1 range,
    2 hard elastic, 3 hard inelastic, 4 hard brems, 5 soft transport."""
    return 4 + 6 * ptype + c


SMP = dict(compton=0, rayleigh=1, moller=2, bhabha=3, brems=4, hard_elastic=5,
           soft=6, pair=7, free_path=8, annih=9, annih_flight=10)
LED_DEP, LED_ESC, LED_POSESC, LED_PATH, LED_EABS, LED_N = range(6)


class Material(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "z_mol", "a_mol", "zz1_mol", "z_screen", "i_exc", "pe_coef", "pe_eref",
        "pe_exp", "pp_coef", "ray_f0", "ray_a", "brems_b")]


class Transport(C.Structure):
    _fields_ = [("n_grid", C.c_int), ("e_min", C.c_double), ("e_max", C.c_double),
                ("eabs", C.c_double * 3), ("c1", C.c_double), ("c2", C.c_double),
                ("wcc", C.c_double), ("wcr", C.c_double), ("flags", C.c_uint32),
                ("force_in", C.c_double), ("force_br", C.c_double), ("split_br", C.c_int)]


class Phantom(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("ox", C.c_double), ("oy", C.c_double), ("oz", C.c_double),
                ("rho", C.POINTER(C.c_double)), ("mat", C.POINTER(C.c_uint8)),
                ("step_cap", C.POINTER(C.c_double))]


class Source(C.Structure):
    _fields_ = [("particle", C.c_int), ("kind", C.c_int), ("energy", C.c_double),
                ("pos", C.c_double * 3), ("dir", C.c_double * 3),
                ("width", C.c_double * 2), ("n_hist", C.c_uint64)]


_STAT_FIELDS = ("histories", "flights", "compton", "photo", "rayleigh", "pair",
                "esteps", "hard_el", "hard_in", "hard_br", "delta", "annih",
                "crossings", "secondaries", "deposits", "absorbed", "escaped")


class Stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in _STAT_FIELDS] + [
        ("e_dep", C.c_double), ("e_esc", C.c_double), ("pos_esc", C.c_uint64), ("maj_excess", C.c_uint64),
        ("annih_flight", C.c_uint64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (FP64, no multiply-add contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-ffp-contract=off",
                               "-fno-fast-math", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        dp = C.POINTER(C.c_double)
        L.orc_tables_create.restype = C.c_void_p
        L.orc_tables_create.argtypes = [C.POINTER(Material), C.POINTER(Transport)]
        L.orc_tables_destroy.argtypes = [C.c_void_p]
        L.orc_eval.restype = C.c_double
        L.orc_eval.argtypes = [C.c_void_p, C.c_int, C.c_double]
        L.orc_node.restype = C.c_double
        L.orc_node.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.orc_node_energy.restype = C.c_double
        L.orc_node_energy.argtypes = [C.c_void_p, C.c_int]
        L.orc_range_inverse.restype = C.c_double
        L.orc_range_inverse.argtypes = [C.c_void_p, C.c_int, C.c_double]
        L.orc_sigma_majorant.restype = C.c_double
        L.orc_sigma_majorant.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double]
        for f in ("orc_screening", "orc_elastic_k"):
            getattr(L, f).restype = C.c_double
            getattr(L, f).argtypes = [C.c_void_p, C.c_double]
        L.orc_mu_cut.restype = C.c_double
        L.orc_mu_cut.argtypes = [C.c_void_p, C.c_int, C.c_double]
        L.orc_soft_a.restype = C.c_double
        L.orc_soft_a.argtypes = [C.c_double]
        L.orc_soft_score.restype = C.c_double
        L.orc_soft_score.argtypes = [C.c_double] * 5
        L.orc_soft_omega2.argtypes = [C.c_void_p, C.c_int, C.c_double]
        L.orc_soft_omega2.restype = C.c_double
        L.orc_sample_straggle.argtypes = [C.c_double, C.c_double, C.c_uint32, C.c_int, dp]
        L.orc_sigma_annih.argtypes = [C.c_void_p, C.c_double]
        L.orc_sigma_annih.restype = C.c_double
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_splitmix64.argtypes = [C.c_uint64]
        L.orc_child_uid.restype = C.c_uint64
        L.orc_child_uid.argtypes = [C.c_uint64, C.c_uint32]
        L.orc_uniforms.argtypes = [C.c_uint32, C.c_uint32, C.c_uint64, C.c_int, dp]
        L.orc_sample.restype = C.c_int
        L.orc_sample.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_uint32, C.c_int, dp, dp]
        L.orc_run.restype = C.c_int
        L.orc_run.argtypes = [C.c_void_p, C.POINTER(Transport), C.POINTER(Phantom),
                              C.POINTER(Source), C.c_int, C.c_uint32, C.c_uint64, C.c_uint64,
                              dp, dp, C.POINTER(Stats), C.POINTER(C.c_uint64), dp]
        L.orc_run_mm.argtypes = [C.c_void_p, C.c_int, C.POINTER(Transport), C.POINTER(Phantom),
                                 C.POINTER(Source), C.c_int, C.c_uint32, C.c_uint64, C.c_uint64,
                                 dp, dp, C.POINTER(Stats), C.POINTER(C.c_uint64), dp]
        L.orc_run_mm.restype = C.c_int
        L.orc_dose.argtypes = [C.POINTER(Phantom), C.c_uint64, dp, dp, dp, dp]
        L.orc_run_gradient.restype = C.c_int
        L.orc_run_gradient.argtypes = [C.c_void_p, C.POINTER(Transport), C.POINTER(Phantom),
                                       C.POINTER(Source), C.c_int, C.c_uint32, C.c_uint64, C.c_uint64,
                                       dp, dp, dp, dp, dp]
        L.orc_run_gradient_mm.restype = C.c_int
        L.orc_run_gradient_mm.argtypes = [C.c_void_p, C.c_int, C.POINTER(Transport), C.POINTER(Phantom),
                                          C.POINTER(Source), C.c_int, C.c_uint32, C.c_uint64, C.c_uint64,
                                          dp, dp, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def material_struct(m: dict) -> Material:
    return Material(**{k: float(m[k]) for k, _ in Material._fields_})


def transport_struct(t: dict) -> Transport:
    s = Transport()
    s.n_grid = int(t["n_grid"])
    s.e_min = float(t["e_min"])
    s.e_max = float(t["e_max"])
    for i in range(3):
        s.eabs[i] = float(t["eabs"][i])
    s.c1, s.c2 = float(t["c1"]), float(t["c2"])
    s.wcc, s.wcr = float(t["wcc"]), float(t["wcr"])
    s.flags = int(t.get("flags", 0))
    s.force_in = float(t.get("force_in", 1.0))
    s.force_br = float(t.get("force_br", 1.0))
    s.split_br = int(t.get("split_br", 1))
    return s


def source_array(sources) -> "C.Array":
    arr = (Source * len(sources))()
    for i, s in enumerate(sources):
        arr[i].particle = int(s["particle"])
        arr[i].kind = int(s["kind"])
        arr[i].energy = float(s["energy"])
        for k in range(3):
            arr[i].pos[k] = float(s["pos"][k])
            arr[i].dir[k] = float(s["dir"][k])
        for k in range(2):
            arr[i].width[k] = float(s.get("width", (0.0, 0.0))[k])
        arr[i].n_hist = int(s["n_hist"])
    return arr


class Tables:
    """Owns one orc_tables handle."""

    def __init__(self, material: dict, transport: dict):
        self.m = material_struct(material)
        self.t = transport_struct(transport)
        self.h = lib().orc_tables_create(C.byref(self.m), C.byref(self.t))
        if not self.h:
            raise ValueError("oracle: invalid material or transport parameters")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_tables_destroy(self.h)
            self.h = None

    def eval(self, ch: int, e: float) -> float:
        return lib().orc_eval(self.h, ch, e)

    def node(self, ch: int, i: int) -> float:
        return lib().orc_node(self.h, ch, i)

    def node_energy(self, i: int) -> float:
        return lib().orc_node_energy(self.h, i)

    def range_inverse(self, ptype: int, r: float) -> float:
        return lib().orc_range_inverse(self.h, ptype, r)

    def majorant(self, ptype: int, elo: float, e: float) -> float:
        return lib().orc_sigma_majorant(self.h, ptype, elo, e)

    def screening(self, e):
        return lib().orc_screening(self.h, e)

    def elastic_k(self, e):
        return lib().orc_elastic_k(self.h, e)

    def mu_cut(self, ptype, e):
        return lib().orc_mu_cut(self.h, ptype, e)

    def soft_omega2(self, ptype: int, e: float) -> float:
        """Second moment of the soft energy-loss DCS per g/cm^2 (MeV^2 cm^2/g)
        of an electron (0) or positron (1)."""
        return lib().orc_soft_omega2(self.h, ptype, e)

    def sigma_annih(self, e: float) -> float:
        """Heitler two-photon annihilation cross section per gram (cm^2/g) of a
        positron of kinetic energy e."""
        return lib().orc_sigma_annih(self.h, e)

    def sample(self, which: str, e: float, n: int, seed: int = 7):
        a = np.zeros(n)
        b = np.zeros(n)
        rc = lib().orc_sample(self.h, SMP[which], e, seed, n, _dp(a), _dp(b))
        if rc:
            raise ValueError(which)
        return a, b


def sample_straggle(m: float, omega2: float, n: int, seed: int = 7) -> np.ndarray:
    """n soft energy losses of mean m and variance omega2 from the Class II
    step's straggling sampler."""
    out = np.zeros(n)
    assert lib().orc_sample_straggle(m, omega2, seed, n, _dp(out)) == 0
    return out


def soft_score(a: float, mu: float, mbar: float, length: float, t1s: float) -> float:
    return lib().orc_soft_score(a, mu, mbar, length, t1s)


def soft_a(mbar: float) -> float:
    return lib().orc_soft_a(mbar)


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def splitmix64(state: int) -> int:
    return lib().orc_splitmix64(state)


def child_uid(uid: int, k: int) -> int:
    return lib().orc_child_uid(uid, k)


def uniforms(seed: int, hist: int, uid: int, n: int) -> np.ndarray:
    out = np.zeros(n)
    lib().orc_uniforms(seed, hist, uid, n, _dp(out))
    return out


def phantom_struct(ph: dict):
    rho = np.ascontiguousarray(ph["rho"], dtype=np.float64).ravel()
    nz, ny, nx = ph["shape"]
    s = Phantom(nx=nx, ny=ny, nz=nz, dx=ph["voxel"][0], dy=ph["voxel"][1], dz=ph["voxel"][2],
                ox=ph["origin"][0], oy=ph["origin"][1], oz=ph["origin"][2], rho=_dp(rho))
    if ph.get("mat") is not None:
        mat = np.ascontiguousarray(ph["mat"], dtype=np.uint8).ravel()
        assert mat.size == rho.size
        s.mat = mat.ctypes.data_as(C.POINTER(C.c_uint8))
        s._keep_mat = mat  # the array must outlive the structure
    if ph.get("step_cap") is not None:
        sc = np.ascontiguousarray(ph["step_cap"], dtype=np.float64).ravel()
        assert sc.size == rho.size
        s.step_cap = _dp(sc)
        s._keep_step_cap = sc
    return s, rho


class RunResult:
    def __init__(self, nvox, n):
        self.sum_q = np.zeros(nvox)
        self.sum_q2 = np.zeros(nvox)
        self.stats = Stats()
        self.n = 0


def run(tables, phantom: dict, sources, seed: int, first: int, n: int,
        result: RunResult | None = None, hashes: bool = False, ledger: bool = False):
    """Transport histories [first, first+n); accumulates into `result`.
    `tables` is one Tables, or a list of Tables (one per material, all on the
    same grid and transport parameters) used with the phantom's "mat"
    array."""
    ph, rho = phantom_struct(phantom)
    nvox = rho.size
    if result is None:
        result = RunResult(nvox, n)
    src = source_array(sources)
    hs = np.zeros(n, dtype=np.uint64) if hashes else None
    led = np.zeros((n, LED_N)) if ledger else None
    hp = hs.ctypes.data_as(C.POINTER(C.c_uint64)) if hs is not None else None
    lp = _dp(led) if led is not None else None
    if isinstance(tables, (list, tuple)):
        arr = (C.c_void_p * len(tables))(*[tb.h for tb in tables])
        rc = lib().orc_run_mm(arr, len(tables), C.byref(tables[0].t), C.byref(ph), src, len(sources), seed, first,
                              n, _dp(result.sum_q), _dp(result.sum_q2), C.byref(result.stats), hp, lp)
    else:
        rc = lib().orc_run(tables.h, C.byref(tables.t), C.byref(ph), src, len(sources), seed, first, n,
                           _dp(result.sum_q), _dp(result.sum_q2), C.byref(result.stats), hp, lp)
    if rc:
        raise RuntimeError(f"orc_run failed: {rc}")
    result.n += n
    result.hashes = hs
    result.ledger = led
    return result


def dose(phantom: dict, result: RunResult, n_hist: int | None = None):
    ph, rho = phantom_struct(phantom)
    d = np.zeros(rho.size)
    s = np.zeros(rho.size)
    lib().orc_dose(C.byref(ph), n_hist or result.n, _dp(result.sum_q), _dp(result.sum_q2), _dp(d), _dp(s))
    shape = tuple(phantom["shape"])
    return d.reshape(shape), s.reshape(shape)


def gradient(tables: Tables, phantom: dict, sources, seed: int, first: int, n: int, dl_ddose: np.ndarray,
             dose: np.ndarray):
    """Score-function estimate of dL/drho for L with dL/dD = dl_ddose (shape of
    the phantom), given the dose D of the same histories (eV/g per history).
    Returns (grad, parts) with parts = dict(a, b, p, qbar) of oracle.h."""
    ph, rho = phantom_struct(phantom)
    vol = phantom["voxel"][0] * phantom["voxel"][1] * phantom["voxel"][2]
    g = np.ascontiguousarray(dl_ddose, dtype=np.float64).ravel()
    w = g * 1e6 / (rho * vol)
    a = np.zeros(rho.size)
    b = np.zeros(rho.size)
    p = np.zeros(rho.size)
    sq = C.c_double(0.0)
    src = source_array(sources)
    if isinstance(tables, (list, tuple)):
        arr = (C.c_void_p * len(tables))(*[tb.h for tb in tables])
        rc = lib().orc_run_gradient_mm(arr, len(tables), C.byref(tables[0].t), C.byref(ph), src, len(sources), seed,
                                       first, n, _dp(w), _dp(a), _dp(b), _dp(p), C.byref(sq))
    else:
        rc = lib().orc_run_gradient(tables.h, C.byref(tables.t), C.byref(ph), src, len(sources), seed, first, n,
                                    _dp(w), _dp(a), _dp(b), _dp(p), C.byref(sq))
    if rc:
        raise RuntimeError(f"orc_run_gradient failed: {rc}")
    qbar = sq.value / n
    grad = (a - qbar * b + p) / n - g * np.asarray(dose, dtype=np.float64).ravel() / rho
    return grad.reshape(tuple(phantom["shape"])), dict(a=a, b=b, p=p, qbar=qbar)
