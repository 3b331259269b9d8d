"""ctypes binding of libkarl (include/karl.h).

Argument marshalling only: every step of the transport runs in the HIP library.  PyTorch
provides the device workspace and the stream.  If libkarl.so is missing the import fails
loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libkarl.so")

MAX_PROC = 16
MAX_SPECIES = 4
NCOUNTERS = 80
NLEDGER = 48
NHIST = 4
NREASON = 9
FP64, FP32 = 0, 1
MAP_AUTO, MAP_LANE, MAP_WAVE = 0, 1, 2
MAPPINGS = {"auto": MAP_AUTO, "lane": MAP_LANE, "wave": MAP_WAVE}
FLAG_DIGESTS, FLAG_HISTORY = 1, 2
# counter and ledger indices (KARL_C_*, KARL_L_* of include/karl.h); per-species entries have
# MAX_SPECIES slots (0 electrons, 1.. ions)
C_BIRTH, C_STEP, C_COLL, C_ZCROSS, C_RCROSS = 0, 4, 8, 12, 16
C_TARGET_REDRAW, C_BEB_TRIES, C_BETA_TRIES, C_PROC, C_DEATH = 20, 21, 22, 24, 40
L_E_PRIMARY, L_E_DEATH, L_E_EXC, L_E_BIND, L_E_GAS, L_T_ALIVE, L_E_FIELD = 0, 1, 37, 38, 39, 40, 44
MOVER_DRIFT, MOVER_BORIS = 0, 1

OK, EINVAL, ENOMEM, EDEVICE, EOVERFLOW, ESTATE, ENUMERIC = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {EINVAL: "KARL_EINVAL", ENOMEM: "KARL_ENOMEM", EDEVICE: "KARL_EDEVICE",
                EOVERFLOW: "KARL_EOVERFLOW", ESTATE: "KARL_ESTATE", ENUMERIC: "KARL_ENUMERIC"}

# names of the entry points declared in include/karl.h
ENTRY_POINTS = ["karl_workspace_bytes", "karl_create_job", "karl_transport",
                "karl_transport_noalloc", "karl_read_tallies",
                "karl_read_fields", "karl_update_target_fields", "karl_reset_tallies",
                "karl_job_stats", "karl_job_drain_stats", "karl_job_slices", "karl_job_mapping",
                "karl_destroy_job",
                "karl_batch_workspace_bytes", "karl_create_batch", "karl_transport_batch",
                "karl_batch_stats", "karl_batch_wave_segments", "karl_destroy_batch",
                "karl_server_workspace_bytes", "karl_create_server", "karl_server_submit",
                "karl_server_step", "karl_server_start", "karl_server_wait", "karl_server_stop",
                "karl_server_poll", "karl_server_job", "karl_server_release",
                "karl_server_stats_get", "karl_destroy_server", "karl_last_error"]


class KarlError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class SpeciesDesc(C.Structure):
    _fields_ = [("mass", C.c_double), ("charge", C.c_double), ("e_cut", C.c_double),
                ("lifetime", C.c_double), ("cap", C.c_int64), ("tracked", C.c_int32),
                ("reserved0", C.c_int32), ("xs_emin", C.c_double), ("xs_emax", C.c_double),
                ("edges", C.POINTER(C.c_double)), ("dens_edges", C.POINTER(C.c_double))]


class ProcessDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("species", C.c_int32), ("target", C.c_int32),
                ("product", C.c_int32), ("partner", C.c_int32), ("density_power", C.c_int32),
                ("e_th", C.c_double), ("xs", C.POINTER(C.c_double)),
                ("ang_bins", C.c_int32), ("ang_nodes", C.c_int32), ("e_iso", C.c_double),
                ("ang_edges", C.POINTER(C.c_double)), ("ang_theta", C.POINTER(C.c_double)),
                ("ang_pdf", C.POINTER(C.c_double))]


class JobDesc(C.Structure):
    _fields_ = [("radius", C.c_double), ("length", C.c_double), ("n_r", C.c_int32),
                ("n_z", C.c_int32), ("n_gas", C.POINTER(C.c_double)),
                ("n_field", C.POINTER(C.c_double) * MAX_SPECIES),
                ("t_gas", C.c_double), ("m_gas", C.c_double),
                ("bz", C.c_double), ("species", SpeciesDesc * MAX_SPECIES),
                ("n_species", C.c_int32), ("n_proc", C.c_int32),
                ("n_e", C.c_int32), ("proc", ProcessDesc * MAX_PROC), ("source", C.c_int32),
                ("beam_species", C.c_int32), ("beta_e0", C.c_double), ("beta_z", C.c_double),
                ("beta_fmax", C.c_double), ("beam_energy", C.c_double),
                ("beam_pos", C.c_double * 3), ("beam_dir", C.c_double * 3),
                ("beam_energy_1", C.c_double),
                ("seed", C.c_uint32), ("n_bins", C.c_int32), ("n_planes", C.c_int32),
                ("reserved0", C.c_int32), ("planes", C.POINTER(C.c_int32)),
                ("n_primaries", C.c_int64), ("precision", C.c_int32), ("flags", C.c_uint32),
                ("queue_capacity", C.c_int64), ("chunk", C.c_int64),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_uint64),
                ("mapping", C.c_int32), ("n_dens_bins", C.c_int32),
                ("mover", C.c_int32), ("reserved1", C.c_int32),
                ("boris_dt", C.c_double * MAX_SPECIES), ("field_nr", C.c_int32),
                ("field_nz", C.c_int32), ("field_radius", C.c_double),
                ("field_length", C.c_double), ("e_field", C.POINTER(C.c_double)),
                ("b_field", C.POINTER(C.c_double)), ("slice_steps", C.c_int64), ("slice_ring", C.c_int64)]


class ServerDesc(C.Structure):
    _fields_ = [("max_jobs", C.c_int32), ("precision", C.c_int32), ("queue_capacity", C.c_int64),
                ("arena_bytes", C.c_uint64), ("round_ms", C.c_double), ("min_quantum", C.c_int64),
                ("max_quantum", C.c_int64), ("n_workers", C.c_int32), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_uint64)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("released", C.c_int64), ("rounds", C.c_int64), ("primaries", C.c_int64),
                ("kernel_ms", C.c_double), ("busy_ms", C.c_double), ("arena_used", C.c_uint64),
                ("arena_peak", C.c_uint64), ("quantum", C.c_int64)]


class Tallies(C.Structure):
    _fields_ = [("counters", C.POINTER(C.c_int64)), ("ledger", C.POINTER(C.c_double)),
                ("density_time", C.POINTER(C.c_double)), ("recomb", C.POINTER(C.c_int64)),
                ("jz", C.POINTER(C.c_int64)), ("jr", C.POINTER(C.c_int64)),
                ("spectra", C.POINTER(C.c_int64)), ("digests", C.POINTER(C.c_uint64)),
                ("hist", C.POINTER(C.c_double)), ("density_time_e", C.POINTER(C.c_double))]


_lib = None


def lib():
    """Load libkarl.so (built by paper_2503_10263_amd.build); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run python -m paper_2503_10263_amd.build "
                               "(hipcc --offload-arch=gfx950); there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        L.karl_workspace_bytes.argtypes = [C.POINTER(JobDesc), C.POINTER(C.c_uint64)]
        L.karl_create_job.argtypes = [C.POINTER(JobDesc), C.POINTER(C.c_void_p)]
        L.karl_transport.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p]
        L.karl_transport_noalloc.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p]
        L.karl_read_tallies.argtypes = [C.c_void_p, C.POINTER(Tallies), C.c_void_p]
        L.karl_read_fields.argtypes = [C.c_void_p, C.c_double, C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p]
        L.karl_update_target_fields.argtypes = [C.c_void_p, C.c_double, C.c_void_p]
        L.karl_reset_tallies.argtypes = [C.c_void_p, C.c_void_p]
        L.karl_job_stats.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.karl_job_slices.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        L.karl_job_drain_stats.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.karl_job_mapping.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_int64)]
        L.karl_destroy_job.argtypes = [C.c_void_p]
        L.karl_batch_workspace_bytes.argtypes = [C.c_int32, C.c_int64, C.POINTER(C.c_uint64)]
        L.karl_create_batch.argtypes = [C.c_int32, C.c_int64, C.c_void_p, C.c_uint64,
                                        C.POINTER(C.c_void_p)]
        L.karl_transport_batch.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                           C.c_int32, C.c_void_p]
        L.karl_batch_stats.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.karl_batch_wave_segments.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        L.karl_destroy_batch.argtypes = [C.c_void_p]
        L.karl_server_workspace_bytes.argtypes = [C.POINTER(ServerDesc), C.POINTER(C.c_uint64)]
        L.karl_create_server.argtypes = [C.POINTER(ServerDesc), C.POINTER(C.c_void_p)]
        L.karl_server_submit.argtypes = [C.c_void_p, C.POINTER(JobDesc), C.POINTER(C.c_int64)]
        L.karl_server_step.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32)]
        L.karl_server_start.argtypes = [C.c_void_p]
        L.karl_server_wait.argtypes = [C.c_void_p, C.c_double, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32)]
        L.karl_server_stop.argtypes = [C.c_void_p]
        L.karl_server_poll.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.c_int32,
                                       C.POINTER(C.c_int32)]
        L.karl_server_job.argtypes = [C.c_void_p, C.c_int64, C.POINTER(C.c_void_p)]
        L.karl_server_release.argtypes = [C.c_void_p, C.c_int64]
        L.karl_server_stats_get.argtypes = [C.c_void_p, C.POINTER(ServerStats)]
        L.karl_destroy_server.argtypes = [C.c_void_p]
        for name in ENTRY_POINTS[:-1]:
            getattr(L, name).restype = C.c_int32
        L.karl_last_error.argtypes = []
        L.karl_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def check(code: int):
    if code != OK:
        raise KarlError(code, lib().karl_last_error().decode(errors="replace"))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Descriptor:
    """karl_job_desc built from a workload; keeps its host arrays alive."""

    def __init__(self, w, precision: int = FP64, flags: int = 0, queue_capacity: int = 0,
                 chunk: int = 0, mapping: int = MAP_AUTO, slice_steps: int = 0, slice_ring: int = 0):
        self.keep = []
        d = JobDesc()
        d.radius, d.length, d.n_r, d.n_z = w.radius, w.length, w.n_r, w.n_z
        d.n_gas = _dptr(self._hold(w.n_gas, np.float64))
        # density fields: slot 0 electrons (n_elec), slot 1 ions (n_ion), further slots from
        # the workload's extra_fields mapping
        fields = {0: getattr(w, "n_elec", None), 1: w.n_ion}
        fields.update(getattr(w, "extra_fields", None) or {})
        for k, f in fields.items():
            if f is not None:
                d.n_field[k] = _dptr(self._hold(f, np.float64))
        d.t_gas, d.m_gas, d.bz = w.t_gas, w.m_gas, w.bz
        nb = len(w.species[0].edges) - 1
        d.n_species = len(w.species)
        for s in range(len(w.species)):
            sp = w.species[s]
            ds = d.species[s]
            ds.mass, ds.charge, ds.e_cut, ds.lifetime = sp.mass, sp.charge, sp.e_cut, sp.lifetime
            ds.cap = int(sp.cap)
            ds.tracked = 1 if sp.tracked else 0
            ds.xs_emin, ds.xs_emax = sp.xs_emin, sp.xs_emax
            edges = self._hold(sp.edges, np.float64)
            if len(edges) != nb + 1:
                raise ValueError("every species needs the same number of spectrum bins")
            ds.edges = _dptr(edges)
            if getattr(w, "dens_edges", None) is not None:
                de = self._hold(w.dens_edges[s], np.float64)
                if len(de) != len(w.dens_edges[0]):
                    raise ValueError("every species needs the same number of density energy bins")
                ds.dens_edges = _dptr(de)
                d.n_dens_bins = len(de) - 1
        d.n_proc = len(w.processes)
        d.n_e = w.n_e
        for i, p in enumerate(w.processes):
            dp = d.proc[i]
            dp.kind, dp.species, dp.target, dp.e_th = p.kind, p.species, p.target, p.e_th
            dp.product = getattr(p, "product", 1)
            partner = getattr(p, "partner", None)
            dp.partner = (1 - p.species) if partner is None else partner
            dp.density_power = getattr(p, "density_power", 1)
            xs = self._hold(p.xs, np.float64)
            if len(xs) != w.n_e:
                raise ValueError(f"process {i}: table has {len(xs)} nodes, expected {w.n_e}")
            dp.xs = _dptr(xs)
            ang = getattr(p, "angular", None)
            if ang is not None:
                edges = self._hold(ang.edges, np.float64)
                theta = self._hold(ang.theta, np.float64)
                pdf = self._hold(ang.pdf, np.float64)
                dp.ang_bins, dp.ang_nodes, dp.e_iso = len(edges) - 1, len(theta), ang.e_iso
                dp.ang_edges, dp.ang_theta, dp.ang_pdf = _dptr(edges), _dptr(theta), _dptr(pdf)
        d.source, d.beam_species = w.source, w.beam_species
        d.beta_e0, d.beta_z, d.beta_fmax = w.beta_e0, w.beta_z, w.beta_fmax
        d.beam_energy = w.beam_energy
        d.beam_energy_1 = getattr(w, "beam_energy_1", 0.0)
        for k in range(3):
            d.beam_pos[k] = w.beam_pos[k]
            d.beam_dir[k] = w.beam_dir[k]
        d.seed = w.seed
        d.n_bins = nb
        planes = self._hold(w.planes, np.int32)
        d.n_planes = len(planes)
        d.planes = planes.ctypes.data_as(C.POINTER(C.c_int32))
        d.n_primaries = w.n_primaries
        d.precision = precision
        d.flags = flags
        d.queue_capacity = queue_capacity
        d.chunk = chunk
        d.mapping = mapping
        d.slice_steps = slice_steps
        d.slice_ring = slice_ring
        # mover and field arrays (one binning shared by E and B)
        d.mover = getattr(w, "mover", MOVER_DRIFT)
        for s, dt in enumerate(getattr(w, "boris_dt", None) or []):
            d.boris_dt[s] = dt
        shapes = set()
        for name in ("e_field", "b_field"):
            arr = getattr(w, name, None)
            if arr is not None:
                a = self._hold(arr, np.float64)
                if a.ndim != 3 or a.shape[2] != 3:
                    raise ValueError(f"{name} must have shape [nr][nz][3]")
                shapes.add(a.shape)
                if len(shapes) > 1:
                    raise ValueError("e_field and b_field share one binning")
                setattr(d, name, _dptr(a))
                d.field_nr, d.field_nz = a.shape[0], a.shape[1]
                d.field_radius, d.field_length = w.field_radius, w.field_length
        self.d = d

    def _hold(self, a, dtype):
        arr = np.ascontiguousarray(np.asarray(a, dtype=dtype))
        self.keep.append(arr)
        return arr

    def workspace_bytes(self) -> int:
        n = C.c_uint64(0)
        check(lib().karl_workspace_bytes(C.byref(self.d), C.byref(n)))
        return int(n.value)


def tally_shapes(w, digests: bool, history: bool) -> Dict[str, tuple]:
    nb = len(w.species[0].edges) - 1
    ns = len(w.species)
    s = {
        "counters": ((NCOUNTERS,), np.int64), "ledger": ((NLEDGER,), np.float64),
        "density_time": ((ns, w.n_r, w.n_z), np.float64), "recomb": ((ns, w.n_r, w.n_z), np.int64),
        "jz": ((ns, w.n_r, w.n_z + 1, 2), np.int64), "jr": ((ns, w.n_r + 1, w.n_z, 2), np.int64),
        "spectra": ((ns, len(w.planes), 2, nb + 2), np.int64),
    }
    if getattr(w, "dens_edges", None) is not None:
        s["density_time_e"] = ((ns, w.n_r, w.n_z, len(w.dens_edges[0]) + 1), np.float64)
    if digests:
        s["digests"] = ((w.n_primaries,), np.uint64)
    if history:
        s["hist"] = ((w.n_primaries, NHIST), np.float64)
    return s


class Job:
    """One transport job on the current HIP device (workspace allocated by torch)."""

    def __init__(self, w, precision: str = "fp64", digests: bool = False, history: bool = False,
                 queue_capacity: int = 0, chunk: int = 0, device=None, mapping: str = "auto",
                 slice_steps: int = 0, slice_ring: int = 0):
        import torch
        self.w = w
        self.precision = FP32 if precision == "fp32" else FP64
        flags = (FLAG_DIGESTS if digests else 0) | (FLAG_HISTORY if history else 0)
        self.digests, self.history = digests, history
        self.desc = Descriptor(w, self.precision, flags, queue_capacity, chunk, MAPPINGS[mapping],
                               slice_steps, slice_ring)
        self.nbytes = self.desc.workspace_bytes()
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=dev)
        self.desc.d.workspace = self.workspace.data_ptr()
        self.desc.d.workspace_bytes = self.nbytes
        h = C.c_void_p()
        with torch.cuda.device(dev):
            check(lib().karl_create_job(C.byref(self.desc.d), C.byref(h)))
        self.h = h

    @staticmethod
    def _stream(stream):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))

    def transport(self, pid_begin: int = 0, pid_end: Optional[int] = None, stream=None):
        if pid_end is None:
            pid_end = self.w.n_primaries
        check(lib().karl_transport(self.h, int(pid_begin), int(pid_end), self._stream(stream)))

    def transport_noalloc(self, pid_begin: int = 0, pid_end: Optional[int] = None, stream=None):
        """karl_transport_noalloc: the same transport with its queues in the library's static
        device array (no allocation during the call)."""
        if pid_end is None:
            pid_end = self.w.n_primaries
        check(lib().karl_transport_noalloc(self.h, int(pid_begin), int(pid_end), self._stream(stream)))

    def read_tallies(self, stream=None, only=None) -> Dict[str, np.ndarray]:
        return _read_tallies(self.h, self.w, self.digests, self.history, stream, only)

    def read_fields(self, activity: float, stream=None) -> Dict[str, np.ndarray]:
        """Densities (m^-3) and currents (m^-2 s^-1) normalised with t_sim = N_prim/activity."""
        return _read_fields(self.h, self.w, activity, stream)

    def update_target_fields(self, activity: float, stream=None):
        """Set each species' target field to its density from the tallies so far (eq. 3-4)."""
        check(lib().karl_update_target_fields(self.h, float(activity), self._stream(stream)))

    def reset(self, stream=None):
        check(lib().karl_reset_tallies(self.h, self._stream(stream)))

    def stats(self) -> Dict[str, float]:
        ms, n, g, q = C.c_double(), C.c_int64(), C.c_int64(), C.c_int64()
        check(lib().karl_job_stats(self.h, C.byref(ms), C.byref(n), C.byref(g), C.byref(q)))
        return {"kernel_ms": ms.value, "launches": n.value, "generations": g.value,
                "max_queue": q.value}

    def drain_stats(self) -> Dict[str, float]:
        """Kernel time and launches of the deferred (drain) launches alone."""
        ms, n = C.c_double(), C.c_int64()
        check(lib().karl_job_drain_stats(self.h, C.byref(ms), C.byref(n)))
        return {"kernel_ms": ms.value, "launches": n.value}

    def slices(self) -> int:
        """Particles put into the ring at the end of a slice by the deferred launches."""
        n = C.c_int64()
        check(lib().karl_job_slices(self.h, C.byref(n)))
        return n.value

    def mapping(self) -> Dict[str, float]:
        """Mapping in use ("auto" until tuned), the segments per interaction that chose it, kernel
        ms per segment of each mapping, segments advanced by wave-cooperative flights."""
        m, r, a, b, n = C.c_int32(), C.c_double(), C.c_double(), C.c_double(), C.c_int64()
        check(lib().karl_job_mapping(self.h, C.byref(m), C.byref(r), C.byref(a), C.byref(b),
                                     C.byref(n)))
        name = {v: k for k, v in MAPPINGS.items()}[m.value]
        return {"mapping": name, "segments_per_interaction": r.value, "ms_per_segment_lane": a.value,
                "ms_per_segment_wave": b.value, "wave_segments": n.value}

    def close(self):
        if getattr(self, "h", None):
            check(lib().karl_destroy_job(self.h))
            self.h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _read_tallies(h, w, digests, history, stream=None, only=None) -> Dict[str, np.ndarray]:
    """karl_read_tallies into fresh arrays; `only` restricts the copy to some of them."""
    shapes = tally_shapes(w, digests, history)
    if only is not None:
        shapes = {k: v for k, v in shapes.items() if k in only}
    out = {k: np.zeros(shp, dt) for k, (shp, dt) in shapes.items()}
    T = Tallies()
    for k, arr in out.items():
        ctype = {np.int64: C.c_int64, np.float64: C.c_double, np.uint64: C.c_uint64}[arr.dtype.type]
        setattr(T, k, arr.ctypes.data_as(C.POINTER(ctype)))
    check(lib().karl_read_tallies(h, C.byref(T), Job._stream(stream)))
    return out


def _read_fields(h, w, activity, stream=None) -> Dict[str, np.ndarray]:
    ns = len(w.species)
    dens = np.zeros((ns, w.n_r, w.n_z))
    jz = np.zeros((ns, w.n_r, w.n_z + 1))
    jr = np.zeros((ns, w.n_r + 1, w.n_z))
    check(lib().karl_read_fields(h, float(activity), _dptr(dens), _dptr(jz), _dptr(jr),
                                 Job._stream(stream)))
    return {"density": dens, "jz": jz, "jr": jr}


class Batch:
    """Secondary queues and job table for launches over many jobs (workspace from torch)."""

    def __init__(self, max_jobs: int, queue_capacity: int = 0, device=None):
        import torch
        n = C.c_uint64(0)
        check(lib().karl_batch_workspace_bytes(int(max_jobs), int(queue_capacity), C.byref(n)))
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.max_jobs = max_jobs
        self.nbytes = int(n.value)
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=dev)
        h = C.c_void_p()
        with torch.cuda.device(dev):
            check(lib().karl_create_batch(int(max_jobs), int(queue_capacity), self.workspace.data_ptr(),
                                          self.nbytes, C.byref(h)))
        self.h = h

    def transport(self, jobs, ranges, stream=None):
        """Transport ranges[i] = (begin, end) of jobs[i] in one sequence of launches."""
        n = len(jobs)
        handles = (C.c_void_p * max(n, 1))(*[j.h for j in jobs])
        flat = (C.c_int64 * max(2 * n, 1))(*[int(x) for r in ranges for x in r])
        check(lib().karl_transport_batch(self.h, handles, flat, n, Job._stream(stream)))

    def stats(self) -> Dict[str, float]:
        ms, n, g, q = C.c_double(), C.c_int64(), C.c_int64(), C.c_int64()
        check(lib().karl_batch_stats(self.h, C.byref(ms), C.byref(n), C.byref(g), C.byref(q)))
        return {"kernel_ms": ms.value, "launches": n.value, "generations": g.value,
                "max_queue": q.value}

    def wave_segments(self) -> int:
        """Flight segments advanced by wave-cooperative flights in this batch's launches."""
        n = C.c_int64()
        check(lib().karl_batch_wave_segments(self.h, C.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "h", None):
            check(lib().karl_destroy_batch(self.h))
            self.h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run(w, pid_begin: int = 0, pid_end: Optional[int] = None, **kw) -> Dict[str, np.ndarray]:
    job = Job(w, **kw)
    try:
        job.transport(pid_begin, pid_end)
        return job.read_tallies()
    finally:
        job.close()


class Server:
    """Continuous batching of transport requests (karl_create_server): jobs are admitted while
    their workspaces fit into an arena of `arena_bytes` device bytes and transported together
    in rounds.  The device memory (batch region + arena) is one torch allocation."""

    def __init__(self, max_jobs: int = 256, arena_bytes: int = 8 << 30, precision: str = "fp32",
                 queue_capacity: int = 0, round_ms: float = 50.0, min_quantum: int = 0,
                 max_quantum: int = 0, n_workers: int = 0, device=None):
        import torch
        self.precision = FP32 if precision == "fp32" else FP64
        d = ServerDesc()
        d.max_jobs, d.precision, d.queue_capacity = int(max_jobs), self.precision, int(queue_capacity)
        d.arena_bytes, d.round_ms = int(arena_bytes), float(round_ms)
        d.min_quantum, d.max_quantum = int(min_quantum), int(max_quantum)
        d.n_workers = int(n_workers)
        n = C.c_uint64(0)
        check(lib().karl_server_workspace_bytes(C.byref(d), C.byref(n)))
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.nbytes = int(n.value)
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=dev)
        d.workspace, d.workspace_bytes = self.workspace.data_ptr(), self.nbytes
        self.d = d
        h = C.c_void_p()
        with torch.cuda.device(dev):
            check(lib().karl_create_server(C.byref(d), C.byref(h)))
        self.h = h
        self.workloads = {}
        self.threaded = False

    def submit(self, w, queue_capacity: int = 256, digests: bool = False) -> int:
        """Queue workload w; the job's own queues stay small (the server's batch holds the
        secondaries).  Returns its ticket."""
        desc = Descriptor(w, self.precision, FLAG_DIGESTS if digests else 0, queue_capacity, 0)
        t = C.c_int64(0)
        check(lib().karl_server_submit(self.h, C.byref(desc.d), C.byref(t)))
        self.workloads[t.value] = w
        return t.value

    def step(self, stream=None):
        """Admit what fits, run one round; returns (n_active, n_pending)."""
        a, p = C.c_int32(0), C.c_int32(0)
        check(lib().karl_server_step(self.h, Job._stream(stream), C.byref(a), C.byref(p)))
        return a.value, p.value

    def start(self):
        """Run admission and rounds in worker threads from now on."""
        check(lib().karl_server_start(self.h))
        self.threaded = True

    def wait(self, timeout_ms: float = 50.0):
        """Wait for a completion (or the timeout); returns (n_active, n_pending)."""
        a, p = C.c_int32(0), C.c_int32(0)
        check(lib().karl_server_wait(self.h, float(timeout_ms), C.byref(a), C.byref(p)))
        return a.value, p.value

    def stop(self):
        check(lib().karl_server_stop(self.h))
        self.threaded = False

    def poll(self, capacity: int = 1024):
        buf = (C.c_int64 * capacity)()
        n = C.c_int32(0)
        check(lib().karl_server_poll(self.h, buf, capacity, C.byref(n)))
        return [buf[i] for i in range(n.value)]

    def _handle(self, ticket: int):
        h = C.c_void_p()
        check(lib().karl_server_job(self.h, int(ticket), C.byref(h)))
        return h

    def read_tallies(self, ticket: int, only=None, stream=None, digests: bool = False) -> Dict[str, np.ndarray]:
        return _read_tallies(self._handle(ticket), self.workloads[ticket], digests, False, stream, only)

    def read_fields(self, ticket: int, activity: float, stream=None) -> Dict[str, np.ndarray]:
        return _read_fields(self._handle(ticket), self.workloads[ticket], activity, stream)

    def release(self, ticket: int):
        check(lib().karl_server_release(self.h, int(ticket)))
        self.workloads.pop(ticket, None)

    def stats(self) -> Dict[str, float]:
        s = ServerStats()
        check(lib().karl_server_stats_get(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            check(lib().karl_destroy_server(self.h))
            self.h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
