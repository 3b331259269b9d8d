"""ctypes front end of the FP64 CPU oracle (karl_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU-baseline
leg of the benchmark, never by the product path.  It shares no code with the HIP
library; it reads a workload description by attribute (duck typing) and packs it
into the oracle's own C structs.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle_karl.so")
SRC = os.path.join(HERE, "karl_oracle.c")

MAX_PROC = 16
MAX_SPECIES = 4
NCOUNTERS = 80
NLEDGER = 48
NHIST = 4
NREASON = 9

# counter / ledger offsets (mirror of karl_oracle.h)
C_BIRTH, C_STEP, C_COLL, C_ZCROSS, C_RCROSS = 0, 4, 8, 12, 16
C_TARGET_REDRAW, C_BEB_TRIES, C_BETA_TRIES = 20, 21, 22
C_PROC, C_DEATH = 24, 40
L_E_PRIMARY, L_E_DEATH, L_E_EXC, L_E_BIND, L_E_GAS, L_T_ALIVE, L_E_FIELD = 0, 1, 37, 38, 39, 40, 44


def build(force: bool = True) -> str:
    """Compile the oracle with every operation rounded once (no contraction)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-Wall",
               "-shared", "-fPIC", "-o", LIB_PATH, SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return LIB_PATH


class _Species(C.Structure):
    _fields_ = [("mass", C.c_double), ("charge", C.c_double), ("e_cut", C.c_double),
                ("lifetime", C.c_double), ("cap", C.c_int64), ("tracked", C.c_int32),
                ("pad", C.c_int32), ("xs_emin", C.c_double), ("xs_emax", C.c_double),
                ("edges", C.POINTER(C.c_double)), ("dens_edges", C.POINTER(C.c_double))]


class _Process(C.Structure):
    _fields_ = [("kind", C.c_int32), ("species", C.c_int32), ("target", C.c_int32),
                ("product", C.c_int32), ("partner", C.c_int32), ("density_power", C.c_int32),
                ("e_th", C.c_double), ("xs", C.POINTER(C.c_double)),
                ("ang_bins", C.c_int32), ("ang_nodes", C.c_int32), ("e_iso", C.c_double),
                ("ang_edges", C.POINTER(C.c_double)), ("ang_theta", C.POINTER(C.c_double)),
                ("ang_pdf", C.POINTER(C.c_double))]


class _Desc(C.Structure):
    _fields_ = [("radius", C.c_double), ("length", C.c_double), ("n_r", C.c_int32),
                ("n_z", C.c_int32), ("n_gas", C.POINTER(C.c_double)),
                ("n_field", C.POINTER(C.c_double) * MAX_SPECIES),
                ("t_gas", C.c_double), ("m_gas", C.c_double),
                ("bz", C.c_double), ("sp", _Species * MAX_SPECIES), ("n_species", C.c_int32),
                ("n_proc", C.c_int32),
                ("n_e", C.c_int32), ("proc", _Process * MAX_PROC), ("source", C.c_int32),
                ("beam_species", C.c_int32), ("beta_e0", C.c_double), ("beta_z", C.c_double),
                ("beta_fmax", C.c_double), ("beam_energy", C.c_double),
                ("beam_pos", C.c_double * 3), ("beam_dir", C.c_double * 3),
                ("beam_energy_1", C.c_double), ("seed", C.c_uint32), ("n_bins", C.c_int32), ("n_planes", C.c_int32),
                ("pad2", C.c_int32), ("planes", C.POINTER(C.c_int32)),
                ("n_primaries", C.c_int64), ("n_dens_bins", C.c_int32), ("mover", C.c_int32),
                ("boris_dt", C.c_double * MAX_SPECIES), ("field_nr", C.c_int32),
                ("field_nz", C.c_int32), ("field_radius", C.c_double),
                ("field_length", C.c_double), ("e_field", C.POINTER(C.c_double)),
                ("b_field", C.POINTER(C.c_double))]


class _Tallies(C.Structure):
    _fields_ = [("counters", C.POINTER(C.c_int64)), ("ledger", C.POINTER(C.c_double)),
                ("density_time", C.POINTER(C.c_double)), ("recomb", C.POINTER(C.c_int64)),
                ("jz", C.POINTER(C.c_int64)), ("jr", C.POINTER(C.c_int64)),
                ("spectra", C.POINTER(C.c_int64)), ("digests", C.POINTER(C.c_uint64)),
                ("hist", C.POINTER(C.c_double)), ("density_time_e", C.POINTER(C.c_double))]


_lib = None
_lib_fast = None


def load_fast() -> C.CDLL:
    """The same source built for speed (-O3 -march=native, contraction allowed) into a
    temporary directory for this host: used only to time the oracle as a CPU baseline, never
    for parity (its results may differ in the last bits)."""
    global _lib_fast
    if _lib_fast is None:
        import tempfile
        out = os.path.join(tempfile.mkdtemp(prefix="karl_oracle_fast_"), "liboracle_karl_fast.so")
        cmd = ["gcc", "-O3", "-march=native", "-std=c99", "-shared", "-fPIC", "-o", out, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        _lib_fast = _setup(C.CDLL(out))
    return _lib_fast


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = _setup(C.CDLL(LIB_PATH))
    return _lib


def _setup(L: C.CDLL) -> C.CDLL:
    L.ko_run.argtypes = [C.POINTER(_Desc), C.c_int64, C.c_int64, C.POINTER(_Tallies)]
    L.ko_run.restype = C.c_int
    L.ko_fields.argtypes = [C.POINTER(_Desc), C.POINTER(_Tallies), C.c_double, C.c_double,
                            C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.ko_fields.restype = C.c_int
    L.ko_philox.argtypes = [C.c_uint32] * 6 + [C.POINTER(C.c_uint32)]
    L.ko_philox.restype = None
    L.ko_u53.argtypes = [C.c_uint32, C.c_uint32]
    L.ko_u53.restype = C.c_double
    L.ko_constants.argtypes = [C.POINTER(C.c_double)]
    L.ko_constants.restype = None
    L.ko_log.argtypes = [C.c_double]
    L.ko_log.restype = C.c_double
    L.ko_sincos.argtypes = [C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.ko_sincos.restype = None
    L.ko_mix64.argtypes = [C.c_uint64]
    L.ko_mix64.restype = C.c_uint64
    L.ko_beta_shape.argtypes = [C.c_double, C.c_double, C.c_double]
    L.ko_beta_shape.restype = C.c_double
    L.ko_birth.argtypes = [C.POINTER(_Desc), C.c_int64, C.POINTER(C.c_double)]
    L.ko_birth.restype = C.c_int
    L.ko_debug_collide.argtypes = [C.POINTER(_Desc), C.c_int, C.c_int64, C.c_uint64,
                                   C.c_uint32, C.c_double, C.POINTER(C.c_double),
                                   C.POINTER(C.c_double)]
    L.ko_debug_collide.restype = C.c_int
    L.ko_debug_angle.argtypes = [C.POINTER(_Desc), C.c_int, C.c_double, C.c_double]
    L.ko_debug_angle.restype = C.c_double
    L.ko_debug_boris.argtypes = [C.POINTER(_Desc), C.c_int, C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_double)]
    L.ko_debug_boris.restype = C.c_int
    L.ko_debug_helix.argtypes = [C.c_double, C.c_double, C.c_double, C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.c_double, C.c_double,
                                 C.POINTER(C.c_double)]
    L.ko_debug_helix.restype = None
    return L


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Desc:
    """Packs a workload into the oracle's descriptor; keeps the numpy buffers alive."""

    def __init__(self, w):
        self.w = w
        self.keep = []
        d = _Desc()
        d.radius = w.radius
        d.length = w.length
        d.n_r = w.n_r
        d.n_z = w.n_z
        n_gas = np.ascontiguousarray(w.n_gas, dtype=np.float64)
        self.keep.append(n_gas)
        d.n_gas = _dptr(n_gas)
        # density fields: slot 0 electrons (n_elec), slot 1 ions (n_ion), further slots from
        # the workload's extra_fields mapping
        flds = {0: getattr(w, "n_elec", None), 1: w.n_ion}
        flds.update(getattr(w, "extra_fields", None) or {})
        for s, f in flds.items():
            if f is not None:
                a = np.ascontiguousarray(f, dtype=np.float64)
                self.keep.append(a)
                d.n_field[s] = _dptr(a)
        d.t_gas = w.t_gas
        d.m_gas = w.m_gas
        d.bz = w.bz
        nb = len(w.species[0].edges) - 1
        d.n_species = len(w.species)
        for s in range(len(w.species)):
            sp = w.species[s]
            edges = np.ascontiguousarray(sp.edges, dtype=np.float64)
            assert len(edges) == nb + 1, "both species need the same number of bins"
            self.keep.append(edges)
            d.sp[s].mass = sp.mass
            d.sp[s].charge = sp.charge
            d.sp[s].e_cut = sp.e_cut
            d.sp[s].lifetime = sp.lifetime
            d.sp[s].cap = int(sp.cap)
            d.sp[s].tracked = 1 if sp.tracked else 0
            d.sp[s].xs_emin = sp.xs_emin
            d.sp[s].xs_emax = sp.xs_emax
            d.sp[s].edges = _dptr(edges)
            if getattr(w, "dens_edges", None) is not None:
                de = np.ascontiguousarray(w.dens_edges[s], dtype=np.float64)
                if len(de) != len(w.dens_edges[0]):
                    raise ValueError("every species needs the same number of density energy bins")
                self.keep.append(de)
                d.sp[s].dens_edges = _dptr(de)
                d.n_dens_bins = len(de) - 1
        d.n_proc = len(w.processes)
        d.n_e = w.n_e
        for i, p in enumerate(w.processes):
            xs = np.ascontiguousarray(p.xs, dtype=np.float64)
            assert len(xs) == w.n_e
            self.keep.append(xs)
            d.proc[i].kind = p.kind
            d.proc[i].species = p.species
            d.proc[i].target = p.target
            d.proc[i].product = getattr(p, "product", 1)
            partner = getattr(p, "partner", None)
            d.proc[i].partner = (1 - p.species) if partner is None else partner
            d.proc[i].density_power = getattr(p, "density_power", 1)
            d.proc[i].e_th = p.e_th
            d.proc[i].xs = _dptr(xs)
            ang = getattr(p, "angular", None)
            if ang is not None:
                edges = np.ascontiguousarray(ang.edges, dtype=np.float64)
                theta = np.ascontiguousarray(ang.theta, dtype=np.float64)
                pdf = np.ascontiguousarray(ang.pdf, dtype=np.float64)
                self.keep += [edges, theta, pdf]
                d.proc[i].ang_bins = len(edges) - 1
                d.proc[i].ang_nodes = len(theta)
                d.proc[i].e_iso = ang.e_iso
                d.proc[i].ang_edges = _dptr(edges)
                d.proc[i].ang_theta = _dptr(theta)
                d.proc[i].ang_pdf = _dptr(pdf)
        d.source = w.source
        d.beam_species = w.beam_species
        d.beta_e0 = w.beta_e0
        d.beta_z = w.beta_z
        d.beta_fmax = w.beta_fmax
        d.beam_energy = w.beam_energy
        d.beam_energy_1 = getattr(w, "beam_energy_1", 0.0)
        for k in range(3):
            d.beam_pos[k] = w.beam_pos[k]
            d.beam_dir[k] = w.beam_dir[k]
        d.seed = w.seed
        d.n_bins = nb
        planes = np.ascontiguousarray(w.planes, dtype=np.int32)
        self.keep.append(planes)
        d.n_planes = len(planes)
        d.planes = planes.ctypes.data_as(C.POINTER(C.c_int32))
        d.n_primaries = w.n_primaries
        # mover and field arrays (Sec. 3.1 "Boris mover"; VectorFieldFromArray)
        d.mover = getattr(w, "mover", 0)
        for s, dt in enumerate(getattr(w, "boris_dt", None) or []):
            d.boris_dt[s] = dt
        shapes = set()
        for name in ("e_field", "b_field"):
            arr = getattr(w, name, None)
            if arr is not None:
                a = np.ascontiguousarray(arr, dtype=np.float64)
                if a.ndim != 3 or a.shape[2] != 3:
                    raise ValueError(f"{name} must have shape [nr][nz][3]")
                shapes.add(a.shape)
                if len(shapes) > 1:
                    raise ValueError("e_field and b_field share one binning")
                self.keep.append(a)
                setattr(d, name, _dptr(a))
                d.field_nr, d.field_nz = a.shape[0], a.shape[1]
                d.field_radius = w.field_radius
                d.field_length = w.field_length
        self.d = d


def empty_tallies(w, digests: bool = False, hist: bool = False) -> Dict[str, np.ndarray]:
    nb = len(w.species[0].edges) - 1
    ns = len(w.species)
    t = {
        "counters": np.zeros(NCOUNTERS, np.int64),
        "ledger": np.zeros(NLEDGER, np.float64),
        "density_time": np.zeros((ns, w.n_r, w.n_z), np.float64),
        "recomb": np.zeros((ns, w.n_r, w.n_z), np.int64),
        "jz": np.zeros((ns, w.n_r, w.n_z + 1, 2), np.int64),
        "jr": np.zeros((ns, w.n_r + 1, w.n_z, 2), np.int64),
        "spectra": np.zeros((ns, len(w.planes), 2, nb + 2), np.int64),
    }
    if digests:
        t["digests"] = np.zeros(w.n_primaries, np.uint64)
    if hist:
        t["hist"] = np.zeros((w.n_primaries, NHIST), np.float64)
    if getattr(w, "dens_edges", None) is not None:
        nd = len(w.dens_edges[0]) - 1
        t["density_time_e"] = np.zeros((ns, w.n_r, w.n_z, nd + 2), np.float64)
    return t


def run(w, pid_begin: int = 0, pid_end: Optional[int] = None, digests: bool = False,
        hist: bool = False, tallies: Optional[Dict[str, np.ndarray]] = None,
        library: Optional[C.CDLL] = None) -> Dict[str, np.ndarray]:
    """Transport primaries [pid_begin, pid_end) of workload `w`; returns (or adds into) tallies.
    `library` selects another build of the same source (load_fast() for timing)."""
    if pid_end is None:
        pid_end = w.n_primaries
    t = tallies if tallies is not None else empty_tallies(w, digests, hist)
    D = Desc(w)
    T = _Tallies()
    T.counters = t["counters"].ctypes.data_as(C.POINTER(C.c_int64))
    T.ledger = _dptr(t["ledger"])
    T.density_time = _dptr(t["density_time"])
    T.recomb = t["recomb"].ctypes.data_as(C.POINTER(C.c_int64))
    T.jz = t["jz"].ctypes.data_as(C.POINTER(C.c_int64))
    T.jr = t["jr"].ctypes.data_as(C.POINTER(C.c_int64))
    T.spectra = t["spectra"].ctypes.data_as(C.POINTER(C.c_int64))
    if "digests" in t:
        T.digests = t["digests"].ctypes.data_as(C.POINTER(C.c_uint64))
    if "hist" in t:
        T.hist = _dptr(t["hist"])
    if "density_time_e" in t:
        T.density_time_e = _dptr(t["density_time_e"])
    rc = (library or lib()).ko_run(C.byref(D.d), pid_begin, pid_end, C.byref(T))
    if rc != 0:
        raise ValueError(f"oracle rejected the job (rc={rc})")
    return t


def _tallies_struct(t):
    T = _Tallies()
    T.counters = t["counters"].ctypes.data_as(C.POINTER(C.c_int64))
    T.ledger = _dptr(t["ledger"])
    T.density_time = _dptr(t["density_time"])
    T.recomb = t["recomb"].ctypes.data_as(C.POINTER(C.c_int64))
    T.jz = t["jz"].ctypes.data_as(C.POINTER(C.c_int64))
    T.jr = t["jr"].ctypes.data_as(C.POINTER(C.c_int64))
    T.spectra = t["spectra"].ctypes.data_as(C.POINTER(C.c_int64))
    if "density_time_e" in t:
        T.density_time_e = _dptr(t["density_time_e"])
    return T


def fields(w, t, n_prim: float, activity: float):
    """Normalised densities and currents from oracle tallies `t` (eqs. 3-5)."""
    D = Desc(w)
    ns = len(w.species)
    dens = np.zeros((ns, w.n_r, w.n_z))
    jz = np.zeros((ns, w.n_r, w.n_z + 1))
    jr = np.zeros((ns, w.n_r + 1, w.n_z))
    T = _tallies_struct(t)
    rc = lib().ko_fields(C.byref(D.d), C.byref(T), n_prim, activity, _dptr(dens), _dptr(jz), _dptr(jr))
    if rc != 0:
        raise ValueError("invalid normalisation arguments")
    return {"density": dens, "jz": jz, "jr": jr}


def philox(k0, k1, c0, c1, c2, c3):
    out = (C.c_uint32 * 4)()
    lib().ko_philox(k0, k1, c0, c1, c2, c3, out)
    return list(out)


def birth(w, pid: int) -> np.ndarray:
    D = Desc(w)
    out = np.zeros(8)
    rc = lib().ko_birth(C.byref(D.d), pid, _dptr(out))
    assert rc == 0
    return out


def collide(w, proc: int, pid: int, lineage: int, s: int, e: float, direction) -> np.ndarray:
    D = Desc(w)
    dr = np.ascontiguousarray(direction, dtype=np.float64)
    out = np.zeros(16)
    rc = lib().ko_debug_collide(C.byref(D.d), proc, pid, lineage, s, e, _dptr(dr), _dptr(out))
    assert rc == 0
    return out


def angle(w, proc: int, e_cm: float, u: float) -> float:
    """Polar centre-of-mass scattering angle of elastic process `proc` (rad)."""
    D = Desc(w)
    return float(lib().ko_debug_angle(C.byref(D.d), int(proc), float(e_cm), float(u)))


def boris(w, sp: int, pos, vel, n: int) -> np.ndarray:
    """n Boris pushes of a particle of species sp (no segments, no interactions):
    position (m) and velocity (m/s)."""
    D = Desc(w)
    x = np.ascontiguousarray(pos, dtype=np.float64)
    v = np.ascontiguousarray(vel, dtype=np.float64)
    out = np.zeros(6)
    rc = lib().ko_debug_boris(C.byref(D.d), int(sp), _dptr(x), _dptr(v), int(n), _dptr(out))
    if rc != 0:
        raise ValueError("oracle rejected the Boris push")
    return out


def helix(charge, mass, bz, pos, direction, speed, path) -> np.ndarray:
    p = np.ascontiguousarray(pos, dtype=np.float64)
    dr = np.ascontiguousarray(direction, dtype=np.float64)
    out = np.zeros(6)
    lib().ko_debug_helix(charge, mass, bz, _dptr(p), _dptr(dr), speed, path, _dptr(out))
    return out


def constants() -> np.ndarray:
    out = np.zeros(6)
    lib().ko_constants(_dptr(out))
    return out


def log(x: float) -> float:
    return lib().ko_log(x)


def sincos(x: float):
    s, c = C.c_double(), C.c_double()
    lib().ko_sincos(x, C.byref(s), C.byref(c))
    return s.value, c.value


def u53(a: int, b: int) -> float:
    return lib().ko_u53(a, b)


def beta_shape(e, e0=18600.0, z=2.0):
    return lib().ko_beta_shape(e, e0, z)
