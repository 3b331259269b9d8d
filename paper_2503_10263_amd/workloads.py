"""Seeded synthetic problem descriptions for the transport hot path.

This module builds the *inputs* of a transport job -- geometry, gas density per
z-cell, target fields, species constants, cross-section tables, spectrum bin
edges and source parameters -- in SI units with energies in eV.  It holds none
of the transport arithmetic (no free-path sampling, kinematics or tallying):
both the HIP library and the oracle consume what it produces.

The paper's own inputs (literature cross sections, the KATRIN gas profile, its
parameter files) are not available, so every table is an analytic placeholder
with the right structure (thresholds, 256 log-spaced nodes, magnitudes of the
electron-H2 and H2+-H2 data shown in the paper's cross-section figures).
Problem statement: geometry and gas profile (Sec. "Density fields",
"Scalar field"), species and processes (Sec. "Interactions", "Species"),
injector (Sec. "Injection"), tallies (Sec. "Density fields",
"Current collection", "Calculation of fields").
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

# ----------------------------------------------------------------------------
# physical constants (CODATA 2018; e and k_B exact by SI definition)
# ----------------------------------------------------------------------------
QE = 1.602176634e-19            # C, also J per eV
KB = 1.380649e-23               # J/K
M_E = 9.1093837015e-31          # kg
AMU = 1.66053906660e-27         # kg
EPS0 = 8.8541878128e-12         # F/m
A0 = 5.29177210903e-11          # Bohr radius, m
RYD_EV = 13.605693122994        # Rydberg energy, eV
M_H2 = 2.01565006414 * AMU      # two 1H atoms (electron masses included)
M_H2P = M_H2 - M_E              # H2+ ion
M_HP = 1.00727646688 * AMU      # proton
M_H3P = 3.0 * 1.00782503207 * AMU - M_E     # H3+ (binding energies neglected)
M_T = 3.01604928 * AMU          # tritium atom
M_T2 = 2.0 * M_T                # T2 molecule (binding energy neglected)
M_TP = M_T - M_E                # T+
M_T2P = M_T2 - M_E              # T2+
M_T3P = 3.0 * M_T - M_E         # T3+

# process kinds
ELASTIC = 0
EXCITATION = 1
IONIZATION = 2
RECOMBINATION = 3
CHARGE_EXCHANGE = 4
CLUSTERING = 5
KIND_NAMES = {ELASTIC: "elastic", EXCITATION: "excitation", IONIZATION: "ionization",
              RECOMBINATION: "recombination", CHARGE_EXCHANGE: "charge exchange",
              CLUSTERING: "clustering"}

# target of a process: the background gas or a density field (Sec. 2.2)
TARGET_GAS = 0
TARGET_FIELD = 1            # the density field of the process's partner species
TARGET_ION_FIELD = TARGET_FIELD

# movers (Sec. 3.1): drift (helix / straight line) or Boris pushes with field arrays
MOVER_DRIFT = 0
MOVER_BORIS = 1

# primary source
SOURCE_BETA = 0
SOURCE_BEAM = 1
SOURCE_PAIR = 2             # beam of both species: even ids electrons, odd ids ions

# species slots: 0 electrons, 1 the molecular ion; chemistry jobs add slots 2 and 3
ELECTRON = 0
ION = 1
MAX_SPECIES = 4

# deletion reasons (deletion logger, Sec. "Termination"); "converted": the projectile of a
# clustering reaction, replaced by its product
REASONS = ["exit_low", "exit_high", "wall", "cutoff", "recombined", "cap",
           "lifetime", "untracked", "converted"]

MAX_PROC = 16

# Upper bound of the unnormalised allowed beta shape used by the rejection
# sampler for E0 = 18600 eV, Z = 2.  The shape's maximum is 1.034917e19 (at
# E = 2499.25 eV, printed by oracle/beta_fmax.py); 1 % headroom.
BETA_E0 = 18600.0
BETA_Z = 2.0
BETA_FMAX = 1.0453e19


@dataclass
class Species:
    """Per-species constants (Sec. "Species": ParticleType -> mass, charge)."""
    name: str
    mass: float                 # kg
    charge: float               # C (signed)
    tracked: bool = True        # False: counted at birth, never transported
    e_cut: float = 0.0          # eV; E < e_cut terminates (strict)
    cap: int = 1_000_000        # maximum number of interactions
    lifetime: float = math.inf  # s
    xs_emin: float = 1.0        # eV, first table node (energy for sigma)
    xs_emax: float = 2.0e4      # eV, last table node
    edges: np.ndarray = field(default_factory=lambda: np.arange(0.0, 2.0e4 + 1.0))


@dataclass
class AngularTable:
    """Scattering-angle distribution of an elastic process (Sec. 3.3 "Elastic scattering"):
    isotropic in the centre-of-mass frame below e_iso, above it a piecewise linear density
    over the polar angle per bin of centre-of-mass impact energy."""
    edges: np.ndarray           # [n_bins+1] eV
    theta: np.ndarray           # [n_nodes] rad, increasing within [0, pi]
    pdf: np.ndarray             # [n_bins][n_nodes] >= 0
    e_iso: float = 0.0          # eV


@dataclass
class Process:
    """One interaction channel (Sec. "Interactions")."""
    kind: int
    species: int                # projectile species slot
    target: int                 # TARGET_GAS or TARGET_FIELD
    e_th: float                 # eV: excitation energy / binding energy; 0 otherwise
    xs: np.ndarray              # [n_e] cross section in m^2 at the species' nodes
    name: str = ""
    angular: Optional[AngularTable] = None   # elastic only; None: isotropic
    product: int = ION          # ionization: ion species made; clustering: species made
    partner: Optional[int] = None   # TARGET_FIELD: species of the field (None: 1 - species)
    density_power: int = 1      # gas targets: rate ~ n_gas^density_power (2: three-body)


@dataclass
class Workload:
    """Complete description of one transport job."""
    name: str
    radius: float               # m
    length: float               # m
    n_r: int
    n_z: int
    n_gas: np.ndarray           # [n_z] m^-3, cell-averaged
    n_ion: Optional[np.ndarray] # [n_r*n_z] m^-3 ion field (target of electrons) or None
    t_gas: float                # K
    m_gas: float                # kg
    bz: float                   # T; 0 selects straight-line transport
    species: List[Species]
    processes: List[Process]
    n_e: int = 256              # table nodes
    source: int = SOURCE_BETA
    beta_e0: float = BETA_E0
    beta_z: float = BETA_Z
    beta_fmax: float = BETA_FMAX
    beam_species: int = ELECTRON
    beam_energy: float = 0.0
    beam_pos: tuple = (0.0, 0.0, 0.0)
    beam_dir: tuple = (0.0, 0.0, 1.0)
    seed: int = 1
    planes: List[int] = field(default_factory=list)   # z-face indices
    n_primaries: int = 0
    n_elec: Optional[np.ndarray] = None   # [n_r*n_z] m^-3 electron field (target of ions)
    dens_edges: Optional[tuple] = None    # per-species energy-bin edges of the density field
    beam_energy_1: float = 0.0            # eV: ion energy of SOURCE_PAIR
    extra_fields: Optional[dict] = None   # slot (2, 3) -> [n_r*n_z] m^-3 density field
    mover: int = MOVER_DRIFT
    boris_dt: Optional[list] = None       # s, per species (Boris mover)
    e_field: Optional[np.ndarray] = None  # [nr][nz][3] (E_r, E_phi, E_z) V/m over the field binning
    b_field: Optional[np.ndarray] = None  # [nr][nz][3] (B_r, B_phi, B_z) T; None: (0, 0, bz)
    field_radius: float = 0.0             # m, extent of the field binning
    field_length: float = 0.0

    @property
    def n_bins(self) -> int:
        return len(self.species[0].edges) - 1

    def describe(self) -> str:
        return (f"{self.name}: R={self.radius} m L={self.length} m grid {self.n_r}x{self.n_z} "
                f"B={self.bz} T procs={len(self.processes)} N={self.n_primaries} seed={self.seed}")


# ----------------------------------------------------------------------------
# table helpers
# ----------------------------------------------------------------------------
def log_nodes(emin: float, emax: float, n: int) -> np.ndarray:
    """Energies of the n log-spaced table nodes (node k at emin*(emax/emin)^(k/(n-1)))."""
    k = np.arange(n, dtype=np.float64)
    return emin * np.exp(k * (math.log(emax / emin) / (n - 1)))


def xs_elastic_e(e: np.ndarray) -> np.ndarray:
    """Placeholder e-H2 elastic cross section (m^2): flat 1.5e-19 at low E, ~E^-1.3 above 20 eV."""
    return 1.5e-19 / (1.0 + (e / 20.0) ** 1.3)


def xs_beb(e: np.ndarray, b: float = 15.43, u: float = 15.98, n: float = 2.0) -> np.ndarray:
    """Kim-Rudd binary-encounter-Bethe total ionization cross section (m^2), zero below B."""
    e = np.asarray(e, dtype=np.float64)
    t = e / b
    uu = u / b
    s = 4.0 * math.pi * A0 * A0 * n * (RYD_EV / b) ** 2
    out = np.zeros_like(e)
    ok = t >= 1.0
    tt = t[ok]
    lt = np.log(tt)
    out[ok] = s / (tt + uu + 1.0) * (0.5 * lt * (1.0 - 1.0 / tt ** 2) + 1.0 - 1.0 / tt - lt / (tt + 1.0))
    return out


def xs_excitation(e: np.ndarray, ex: float, amp: float) -> np.ndarray:
    """Placeholder excitation shape amp*(1-x)*ln(1/x+1)*x with x = ex/E, zero below ex."""
    e = np.asarray(e, dtype=np.float64)
    out = np.zeros_like(e)
    ok = e > ex
    x = ex / e[ok]
    out[ok] = amp * (1.0 - x) * np.log(1.0 / x + 1.0) * x
    return out


def xs_recombination(e: np.ndarray) -> np.ndarray:
    """Placeholder radiative recombination cross section 1e-21 m^2 * (1 eV / E)."""
    return 1.0e-21 / np.asarray(e, dtype=np.float64)


def xs_langevin(e_cm: np.ndarray, alpha_vol: float = 0.787e-30) -> np.ndarray:
    """Langevin capture cross section pi*sqrt(2 a' e^2/(4 pi eps0 E_cm)) (m^2), E_cm in eV."""
    e2 = QE * QE / (4.0 * math.pi * EPS0)
    return math.pi * np.sqrt(2.0 * alpha_vol * e2 / (np.asarray(e_cm) * QE))


def cell_average(knots_z, knots_v, length: float, n_z: int) -> np.ndarray:
    """Exact cell averages of a piecewise-linear profile over n_z equal cells."""
    kz = np.asarray(knots_z, dtype=np.float64)
    kv = np.asarray(knots_v, dtype=np.float64)
    out = np.empty(n_z)
    dz = length / n_z
    for k in range(n_z):
        a, b = k * dz, (k + 1) * dz
        pts = np.concatenate(([a], kz[(kz > a) & (kz < b)], [b]))
        vals = np.interp(pts, kz, kv)
        out[k] = np.sum(0.5 * (vals[1:] + vals[:-1]) * np.diff(pts)) / (b - a)
    return out


def electron(e_cut=1.0, cap=1_000_000, edges=None, emin=1.0, emax=2.0e4) -> Species:
    return Species("e-", M_E, -QE, True, e_cut, cap, math.inf, emin, emax,
                   np.arange(0.0, 2.0e4 + 1.0) if edges is None else np.asarray(edges, np.float64))


def h2_ion(tracked: bool, cap=1_000_000, edges=None, emin=1.0e-4, emax=1.0e2, n_bins=20000) -> Species:
    if edges is None:
        edges = np.linspace(0.0, 100.0, n_bins + 1)
    return Species("H2+", M_H2P, QE, tracked, 0.0, cap, math.inf, emin, emax, np.asarray(edges, np.float64))


def _cfg1_processes(n_e: int) -> List[Process]:
    en = log_nodes(1.0, 2.0e4, n_e)
    return [
        Process(ELASTIC, ELECTRON, TARGET_GAS, 0.0, xs_elastic_e(en), "e elastic"),
        Process(IONIZATION, ELECTRON, TARGET_GAS, 15.43, xs_beb(en), "e ionization (BEB)"),
        Process(EXCITATION, ELECTRON, TARGET_GAS, 12.6, xs_excitation(en, 12.6, 1.5e-20), "e exc 12.6"),
    ]


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------
# Launch configuration of the measured runs.  Full case: primaries per transport call, one
# chunk, so that the call's H2+ run in one deferred launch of about five ion lifetimes per
# lane; that launch in slices of 2^15 steps (about half a second of an ion's 12 s), so that the
# long histories end together.  Batched case: queue entries (76 GB of HBM), so that its 256 jobs
# run in a few chunks with few generation launches.
FULL_STEP_PRIMARIES = 131072
FULL_SLICE_STEPS = 1 << 15
BATCHED_QUEUE = 1 << 28


def cfg_tiny(n_primaries: int = 10_000, seed: int = 1, bz: float = 0.0,
             column_cm2: float = 1.0e16, n_r: int = 1, n_z: int = 1, n_e: int = 256) -> Workload:
    """Tiny plain FP64 case: 1 m tube of radius 45 mm, uniform H2 with the given column
    density, straight-line transport, elastic + BEB ionization + one 12.6 eV excitation,
    1 eV exit spectra at both ends; ions counted, not tracked.  Cross-section tables of n_e
    log-spaced nodes (256 in the case itself)."""
    length = 1.0
    n = column_cm2 * 1.0e4 / length
    return Workload(
        name="tiny", radius=0.045, length=length, n_r=n_r, n_z=n_z,
        n_gas=np.full(n_z, n), n_ion=None, t_gas=80.0, m_gas=M_H2, bz=bz,
        species=[electron(), h2_ion(tracked=False)], processes=_cfg1_processes(n_e),
        n_e=n_e, source=SOURCE_BETA, seed=seed, planes=[0, n_z], n_primaries=n_primaries)


def cfg_full(n_primaries: int = 1_000_000, seed: int = 1, n_e: int = 256) -> Workload:
    """Full plain FP64 case: 10 m cylinder of radius 45 mm, axial profile flat over the
    central 8 m with linear falloff to 5 % at the ends (column 5e17 cm^-2), uniform 2.5 T
    axial field (guiding-centre transport), 8 electron processes including recombination on
    a frozen ion-density field, tracked H2+ with Langevin elastic scattering, 64x512 (r,z)
    grids and 2048-bin spectra per species at z = 0, 5, 10 m.  Cross-section tables of n_e
    log-spaced nodes (256 in the case itself)."""
    length, n_z, n_r = 10.0, 512, 64
    column = 5.0e17 * 1.0e4
    shape = cell_average([0.0, 1.0, 9.0, 10.0], [0.05, 1.0, 1.0, 0.05], length, n_z)
    n0 = column / (9.05)            # integral of the shape over 10 m is 9.05 m
    n_gas = n0 * shape
    n_ion = np.repeat((1.0e15 * shape)[None, :], n_r, axis=0).reshape(-1)
    en = log_nodes(1.0, 2.0e4, n_e)
    ei = log_nodes(1.0e-4, 1.0e2, n_e)
    procs = [
        Process(ELASTIC, ELECTRON, TARGET_GAS, 0.0, xs_elastic_e(en), "e elastic"),
        Process(IONIZATION, ELECTRON, TARGET_GAS, 15.43, xs_beb(en), "e ionization (BEB)"),
        Process(EXCITATION, ELECTRON, TARGET_GAS, 8.9, xs_excitation(en, 8.9, 1.5e-20), "e exc 8.9"),
        Process(EXCITATION, ELECTRON, TARGET_GAS, 11.37, xs_excitation(en, 11.37, 1.5e-20), "e exc 11.37"),
        Process(EXCITATION, ELECTRON, TARGET_GAS, 12.6, xs_excitation(en, 12.6, 1.5e-20), "e exc 12.6"),
        Process(EXCITATION, ELECTRON, TARGET_GAS, 0.516, xs_excitation(en, 0.516, 3.0e-21), "e vib 0.516"),
        Process(EXCITATION, ELECTRON, TARGET_GAS, 0.044, xs_excitation(en, 0.044, 5.0e-21), "e rot 0.044"),
        Process(RECOMBINATION, ELECTRON, TARGET_ION_FIELD, 0.0, xs_recombination(en), "e recombination"),
        Process(ELASTIC, ION, TARGET_GAS, 0.0, xs_langevin(ei), "H2+ Langevin elastic"),
    ]
    e_edges = 1.0 * (2.0e4 / 1.0) ** (np.arange(2049) / 2048.0)
    i_edges = 1.0e-4 * (1.0e2 / 1.0e-4) ** (np.arange(2049) / 2048.0)
    return Workload(
        name="full", radius=0.045, length=length, n_r=n_r, n_z=n_z, n_gas=n_gas, n_ion=n_ion,
        t_gas=80.0, m_gas=M_H2, bz=2.5,
        species=[electron(edges=e_edges), h2_ion(tracked=True, edges=i_edges)],
        processes=procs, n_e=n_e, source=SOURCE_BETA, seed=seed,
        planes=[0, 256, 512], n_primaries=n_primaries)


def cfg_batched(n_jobs: int = 256, rng_seed: int = 20250313, scale: float = 1.0) -> List[Workload]:
    """Batched case: n_jobs jobs with tiny-case physics in guiding-centre mode; primaries
    log-uniform in 1e3-1e6 (times `scale`), column log-uniform in 1e16-1e18 cm^-2 over 1 m,
    B uniform in 1-3.6 T, Philox seed 1000+j."""
    rng = np.random.default_rng(rng_seed)
    jobs = []
    for j in range(n_jobs):
        n_prim = int(round(10.0 ** rng.uniform(3.0, 6.0) * scale))
        column = 10.0 ** rng.uniform(16.0, 18.0)
        b = float(rng.uniform(1.0, 3.6))
        w = cfg_tiny(n_primaries=max(n_prim, 1), seed=1000 + j, bz=b, column_cm2=column)
        w.name = f"batched[{j}]"
        jobs.append(w)
    return jobs


def cfg_mixed(n_primaries: int = 100_000_000, seed: int = 1) -> Workload:
    """Mixed-precision case: tiny-case geometry and physics at 1e8 primaries."""
    w = cfg_tiny(n_primaries=n_primaries, seed=seed)
    w.name = "mixed"
    return w


def serving_requests(n: int = 600, rate: float = 20.0, rng_seed: int = 20250313,
                     scale: float = 1.0):
    """Serving case: Poisson arrivals at `rate` jobs/s; each job a tiny-case variant in
    guiding-centre mode with column 1e16-1e18 cm^-2, B 1-3.6 T, primaries log-uniform
    1e4-1e7 (times `scale`), grid 32x256, 48x384 or 64x512.  Returns (arrival_s, Workload)."""
    rng = np.random.default_rng(rng_seed)
    t = 0.0
    out = []
    grids = [(32, 256), (48, 384), (64, 512)]
    for j in range(n):
        t += rng.exponential(1.0 / rate)
        column = 10.0 ** rng.uniform(16.0, 18.0)
        b = float(rng.uniform(1.0, 3.6))
        n_prim = int(round(10.0 ** rng.uniform(4.0, 7.0) * scale))
        n_r, n_z = grids[int(rng.integers(0, 3))]
        w = cfg_tiny(n_primaries=max(n_prim, 1), seed=5000 + j, bz=b, column_cm2=column,
                     n_r=n_r, n_z=n_z)
        w.name = f"serve[{j}]"
        out.append((t, w))
    return out


# ----------------------------------------------------------------------------
# small test problems (beams, single processes)
# ----------------------------------------------------------------------------
def beam_problem(energy: float, processes: List[Process], n_gas: np.ndarray, length: float,
                 radius: float = 1.0, n_r: int = 1, bz: float = 0.0, t_gas: float = 0.0,
                 n_primaries: int = 10_000, seed: int = 7, species: Optional[List[Species]] = None,
                 planes: Optional[List[int]] = None, n_ion: Optional[np.ndarray] = None,
                 beam_pos=(0.0, 0.0, 0.0), beam_dir=(0.0, 0.0, 1.0), beam_species: int = ELECTRON,
                 n_e: int = 256) -> Workload:
    """A directed mono-energetic beam (Sec. "Injection": directed streams for tests)."""
    n_z = len(n_gas)
    if species is None:
        species = [electron(), h2_ion(tracked=False)]
    return Workload(
        name="beam", radius=radius, length=length, n_r=n_r, n_z=n_z,
        n_gas=np.asarray(n_gas, np.float64), n_ion=n_ion, t_gas=t_gas, m_gas=M_H2, bz=bz,
        species=species, processes=processes, n_e=n_e, source=SOURCE_BEAM,
        beam_species=beam_species, beam_energy=energy, beam_pos=tuple(beam_pos),
        beam_dir=tuple(beam_dir), seed=seed, planes=[0, n_z] if planes is None else planes,
        n_primaries=n_primaries)


def recombination_pair(sigma_e: float, sigma_i: float, n_primaries: int = 20000, n_z: int = 40,
                       length: float = 1.0, radius: float = 0.05, e_electron: float = 2.0,
                       seed: int = 11, n_elec: Optional[np.ndarray] = None,
                       n_ion: Optional[np.ndarray] = None) -> Workload:
    """Electrons and H2+ ions injected together on the axis at z = 0 along +z with equal speeds
    (ion energy = electron energy x M/m), no gas: the only process of each species is
    recombination with the density field of the other (constant cross sections sigma_e,
    sigma_i).  The coupled steady state of Sec. 4 "Recombination" (both partners variable)."""
    e_ion = e_electron * M_H2P / M_E
    species = [electron(e_cut=0.0, emin=1.0e-3, emax=2.0e4, edges=np.linspace(0.0, 10.0, 11)),
               Species("H2+", M_H2P, QE, True, 0.0, 1_000_000, math.inf, 1.0e-3, 2.0e4,
                       np.linspace(0.0, 1.0e4, 11))]
    procs = [Process(RECOMBINATION, ELECTRON, TARGET_FIELD, 0.0, np.full(64, sigma_e), "e recombination"),
             Process(RECOMBINATION, ION, TARGET_FIELD, 0.0, np.full(64, sigma_i), "ion recombination")]
    return Workload(
        name="recombination pair", radius=radius, length=length, n_r=1, n_z=n_z,
        n_gas=np.zeros(n_z), n_ion=n_ion, t_gas=0.0, m_gas=M_H2, bz=0.0, species=species,
        processes=procs, n_e=64, source=SOURCE_PAIR, beam_species=ELECTRON,
        beam_energy=e_electron, beam_energy_1=e_ion, beam_pos=(0.0, 0.0, 0.0),
        beam_dir=(0.0, 0.0, 1.0), seed=seed, planes=[0, n_z], n_primaries=n_primaries,
        n_elec=n_elec)


def screened_table(e_iso: float = 100.0, n_bins: int = 6, n_nodes: int = 64,
                   emin: float = 100.0, emax: float = 2.0e4) -> AngularTable:
    """A composite elastic distribution like the paper's electron case: isotropic below e_iso,
    above it a forward-peaked screened-Rutherford shape p(theta) ~ sin(theta) / (1 + 2 eta -
    cos(theta))^2 with screening eta = 3.4 eV / E (stronger forward peak at higher energy),
    tabulated at the centre of each log-spaced energy bin on nodes denser near 0."""
    edges = np.geomspace(emin, emax, n_bins + 1)
    theta = np.pi * np.linspace(0.0, 1.0, n_nodes) ** 2
    pdf = np.zeros((n_bins, n_nodes))
    for b in range(n_bins):
        e = math.sqrt(edges[b] * edges[b + 1])
        eta = 3.4 / e
        pdf[b] = np.sin(theta) / (1.0 + 2.0 * eta - np.cos(theta)) ** 2
    return AngularTable(edges=edges, theta=theta, pdf=pdf, e_iso=e_iso)


# ----------------------------------------------------------------------------
# ion chemistry (Sec. 3.3 "Clustering", "Charge exchange", "Ionization";
# Sec. 4 "Clustering", "Charge Exchange")
# ----------------------------------------------------------------------------
def rate_table(k: float, mass: float, m_gas: float, nodes_xs: np.ndarray) -> np.ndarray:
    """Cross section k / v of a process known by its rate coefficient k (m^3/s for two-body,
    m^6/s for three-body reactions, giving m^2 or m^5), at table nodes given as the
    interpolation energy E_xs = E M/(m+M) of a projectile of `mass` on gas at rest; v is the
    projectile's speed at E = E_xs (m+M)/M."""
    e_lab = np.asarray(nodes_xs, np.float64) * (mass + m_gas) / m_gas
    v = np.sqrt(2.0 * e_lab * QE / mass)
    return k / v


def xs_charge_exchange(e_cm: np.ndarray, a: float = 4.0e-10, b: float = 0.3e-10) -> np.ndarray:
    """Resonant charge-exchange shape sigma = (a - b ln(E/eV))^2 (m^2), E in eV."""
    return (a - b * np.log(np.asarray(e_cm, np.float64))) ** 2


def ion_species(name: str, mass: float, tracked: bool = True, emin: float = 1.0e-4,
                emax: float = 1.0e2, n_bins: int = 100, lifetime: float = math.inf) -> Species:
    return Species(name, mass, QE, tracked, 0.0, 1_000_000, lifetime, emin, emax,
                   np.linspace(0.0, emax, n_bins + 1))


CLUSTERING_CASES = {
    # name: (projectile slot, density (m^-3), density power, cross section or rate coefficient)
    "t2p_radiative": (ION, 1.0e18, 1, 1.91e-18),     # T2+ + T2 -> T3+ + T, sigma (m^2)
    "tp_tertiary": (2, 1.0e22, 2, 2.6e-41),          # T+ + 2 T2 -> T3+ + T2, k_ter (m^6/s)
    "tp_radiative": (2, 2.0e25, 1, 5.0e-23),         # T+ + T2 -> T3+ + h nu, k_rad (m^3/s)
}


def clustering_beam(case: str, n_primaries: int = 80_000, e_beam: float = 6.8e-3,
                    length: float = 2.0, n_z: int = 40, bz: float = 2.5, t_gas: float = 80.0,
                    seed: int = 21) -> Workload:
    """The clustering test of Sec. 4: an ion beam of 6.8 meV along +z on the axis of a uniform
    tritium column in a 2.5 T field; the only process of the injected ion is clustering into
    T3+ (slot 3), with the paper's cross section (T2+) or rate coefficient (T+ radiative and
    three-body, 80 K values).  Species: e- (0), T2+ (1), T+ (2), T3+ (3, no processes).  The
    injected ion's density decays as exp(-z / lambda) with lambda = 1/(sigma n), v/(k n) or
    v/(k n^2)."""
    slot, n, power, coef = CLUSTERING_CASES[case]
    masses = {ION: M_T2P, 2: M_TP}
    m = masses[slot]
    n_e = 64
    gf = M_T2 / (m + M_T2)
    e_xs = e_beam * gf
    # table nodes from the beam's interpolation energy upwards: the beam sits on node 0
    ions = []
    for name, mass in (("T2+", M_T2P), ("T+", M_TP), ("T3+", M_T3P)):
        ions.append(ion_species(name, mass, emin=e_xs if mass == m else 1.0e-4, emax=1.0e2))
    nodes = log_nodes(e_xs, 1.0e2, n_e)
    xs = np.full(n_e, coef) if case == "t2p_radiative" else rate_table(coef, m, M_T2, nodes)
    proc = [Process(CLUSTERING, slot, TARGET_GAS, 0.0, xs, case, product=3, density_power=power)]
    species = [electron(edges=np.linspace(0.0, 2.0e4, 11)), *ions]
    for sp in ions:
        sp.edges = np.linspace(0.0, 1.0, 11)
    return Workload(
        name=f"clustering {case}", radius=0.05, length=length, n_r=1, n_z=n_z,
        n_gas=np.full(n_z, n), n_ion=None, t_gas=t_gas, m_gas=M_T2, bz=bz, species=species,
        processes=proc, n_e=n_e, source=SOURCE_BEAM, beam_species=slot, beam_energy=e_beam,
        beam_pos=(0.0, 0.0, 0.0), beam_dir=(0.0, 0.0, 1.0), seed=seed, planes=[0, n_z],
        n_primaries=n_primaries)


def charge_exchange_box(n_primaries: int = 2000, e_beam: float = 10.0, n: float = 1.224e19,
                        t_gas: float = 80.0, lifetime: float = 0.5, n_bins: int = 40,
                        seed: int = 23) -> Workload:
    """The charge-exchange test of Sec. 4 in an unbounded form: T2+ ions of 10 eV start in a T2
    gas of 1.224e19 m^-3 at 80 K whose only ion process is resonant charge exchange; the
    column (1 km) is far larger than the ions' diffusion length and every ion is deleted
    after `lifetime`, so the time spent per energy interval (the energy-resolved density
    field) tends to the Maxwell-Boltzmann energy density of the gas, weighted with the mean
    time between exchanges, 1/(n sigma(E) v(E))."""
    n_e = 256
    emin, emax = 1.0e-5, 1.0e2
    nodes = log_nodes(emin, emax, n_e)
    proc = [Process(CHARGE_EXCHANGE, ION, TARGET_GAS, 0.0, xs_charge_exchange(nodes),
                    "T2+ charge exchange")]
    ion = ion_species("T2+", M_T2P, emin=emin, emax=emax, n_bins=n_bins, lifetime=lifetime)
    species = [electron(edges=np.linspace(0.0, 2.0e4, n_bins + 1)), ion]
    kt = KB * t_gas / QE
    e_hi = 8.0 * kt * M_T2P / M_T2
    edges = np.linspace(0.0, e_hi, n_bins + 1)
    w = Workload(
        name="charge exchange", radius=1.0e3, length=2.0e3, n_r=1, n_z=1,
        n_gas=np.array([n]), n_ion=None, t_gas=t_gas, m_gas=M_T2, bz=0.0, species=species,
        processes=proc, n_e=n_e, source=SOURCE_BEAM, beam_species=ION, beam_energy=e_beam,
        beam_pos=(0.0, 0.0, 1.0e3), beam_dir=(0.0, 0.0, 1.0), seed=seed, planes=[0, 1],
        n_primaries=n_primaries)
    w.dens_edges = (np.linspace(0.0, 2.0e4, n_bins + 1), edges)
    return w


def hydrogen_chemistry(n_primaries: int = 4000, bz: float = 2.5, column_cm2: float = 5.0e15,
                       n_r: int = 4, n_z: int = 32, seed: int = 31,
                       boost: float = 1.0e6) -> Workload:
    """Beta electrons in H2 with the ion chemistry of Sec. 3.3 on the same kernels: electron
    elastic scattering, excitation, ionization to H2+ (slot 1) and dissociative ionization to
    H+ (slot 2); H2+ elastic scattering, charge exchange and clustering to H3+ (slot 3); H+
    elastic scattering with radiative and three-body clustering to H3+; H3+ elastic
    scattering; H+ recombining on the electron field and electrons on the H3+ field.  The
    clustering rate coefficients are the paper's 80 K values times `boost` and the
    recombination cross sections are enlarged likewise, so that a short tube sees all
    channels."""
    n_e = 256
    length = 1.0
    n = column_cm2 * 1.0e4 / length
    en = log_nodes(1.0, 2.0e4, n_e)
    ei = log_nodes(1.0e-4, 1.0e2, n_e)
    procs = [
        Process(ELASTIC, ELECTRON, TARGET_GAS, 0.0, xs_elastic_e(en), "e elastic"),
        Process(IONIZATION, ELECTRON, TARGET_GAS, 15.43, xs_beb(en), "e ionization -> H2+",
                product=ION),
        Process(IONIZATION, ELECTRON, TARGET_GAS, 18.08, 0.1 * xs_beb(en, b=18.08, u=18.08),
                "e dissociative ionization -> H+", product=2),
        Process(EXCITATION, ELECTRON, TARGET_GAS, 12.6, xs_excitation(en, 12.6, 1.5e-20), "e exc 12.6"),
        Process(RECOMBINATION, ELECTRON, TARGET_FIELD, 0.0, 1.0e5 * xs_recombination(en),
                "e + H3+ recombination", partner=3),
        Process(ELASTIC, ION, TARGET_GAS, 0.0, xs_langevin(ei), "H2+ Langevin elastic"),
        Process(CHARGE_EXCHANGE, ION, TARGET_GAS, 0.0, xs_charge_exchange(ei), "H2+ charge exchange"),
        Process(CLUSTERING, ION, TARGET_GAS, 0.0, np.full(n_e, 1.91e-18), "H2+ + H2 -> H3+ + H",
                product=3),
        Process(ELASTIC, 2, TARGET_GAS, 0.0, xs_langevin(ei), "H+ Langevin elastic"),
        Process(CLUSTERING, 2, TARGET_GAS, 0.0, rate_table(5.0e-23 * boost, M_HP, M_H2, ei),
                "H+ + H2 -> H3+ radiative", product=3),
        Process(CLUSTERING, 2, TARGET_GAS, 0.0, rate_table(2.6e-41 * boost, M_HP, M_H2, ei),
                "H+ + 2 H2 -> H3+ three-body", product=3, density_power=2),
        Process(RECOMBINATION, 2, TARGET_FIELD, 0.0, np.full(n_e, 2.0e-16), "H+ + e recombination",
                partner=ELECTRON),
        Process(ELASTIC, 3, TARGET_GAS, 0.0, xs_langevin(ei), "H3+ Langevin elastic"),
    ]
    z = (np.arange(n_z) + 0.5) / n_z
    n_e_field = np.repeat((2.0e15 * (1.0 - 0.5 * z))[None, :], n_r, axis=0).reshape(-1)
    n_h3_field = np.repeat((1.0e15 * (0.5 + z))[None, :], n_r, axis=0).reshape(-1)
    species = [electron(),
               ion_species("H2+", M_H2P, n_bins=200),
               ion_species("H+", M_HP, n_bins=200),
               ion_species("H3+", M_H3P, n_bins=200)]
    species[0].edges = np.linspace(0.0, 2.0e4, 201)
    return Workload(
        name="hydrogen chemistry", radius=0.045, length=length, n_r=n_r, n_z=n_z,
        n_gas=np.full(n_z, n), n_ion=None, t_gas=80.0, m_gas=M_H2, bz=bz, species=species,
        processes=procs, n_e=n_e, source=SOURCE_BETA, seed=seed, planes=[0, n_z // 2, n_z],
        n_primaries=n_primaries, n_elec=n_e_field, extra_fields={3: n_h3_field})


def uniform_vector_field(nr: int, nz: int, vec_cyl) -> np.ndarray:
    """[nr][nz][3] array holding the same (r, phi, z) components in every bin."""
    return np.tile(np.asarray(vec_cyl, np.float64), (nr, nz, 1))


def with_boris(w: Workload, dt, lifetime, e_field=None, b_field=None, field_radius=None,
               field_length=None) -> Workload:
    """Switch a workload to the Boris mover (Sec. 3.1): time step and (finite) lifetime per
    species, optional field arrays over a cylindrical binning (default: the job's cylinder)."""
    w.mover = MOVER_BORIS
    w.boris_dt = list(dt)
    for sp, life in zip(w.species, lifetime):
        sp.lifetime = life
    w.e_field, w.b_field = e_field, b_field
    w.field_radius = w.radius if field_radius is None else field_radius
    w.field_length = w.length if field_length is None else field_length
    return w


def boris_column(n_primaries: int = 600, column_cm2: float = 2.0e15, n_r: int = 4, n_z: int = 16,
                 b0: float = 0.05, b_max: float = 0.1, e_r: float = -30.0, seed: int = 51,
                 field_bins: tuple = (8, 32)) -> Workload:
    """Beta electrons and tracked H2+ moved by Boris pushes (Sec. 3.1) in a 1 m x 45 mm H2
    column through a magnetic bottle B_z(z) = b0 + (b_max - b0)(2z/L - 1)^2 with
    B_r = -(r/2) dB_z/dz at the bin centres and a radial electric field E_r = e_r (r/R) V/m
    (arrays over field_bins (r, z) bins).  Electrons: elastic, BEB ionization, 12.6 eV
    excitation; ions: Langevin elastic.  Time steps 2e-11 s (electrons; the largest gyro
    frequency is 1.8e10 rad/s) and 1e-7 s (ions), lifetimes 2e-6 s and 2e-4 s."""
    w = cfg_tiny(n_primaries=n_primaries, seed=seed, bz=0.0, column_cm2=column_cm2, n_r=n_r, n_z=n_z)
    w.name = "boris column"
    w.species[ION] = h2_ion(tracked=True, edges=np.linspace(0.0, 100.0, 20001))
    w.processes.append(Process(ELASTIC, ION, TARGET_GAS, 0.0,
                               xs_langevin(log_nodes(1.0e-4, 1.0e2, w.n_e)), "H2+ Langevin elastic"))
    nfr, nfz = field_bins
    zc = (np.arange(nfz) + 0.5) / nfz * w.length
    rc = (np.arange(nfr) + 0.5) / nfr * w.radius
    bz = b0 + (b_max - b0) * (2.0 * zc / w.length - 1.0) ** 2
    dbz = (b_max - b0) * 2.0 * (2.0 * zc / w.length - 1.0) * (2.0 / w.length)
    b = np.zeros((nfr, nfz, 3))
    b[:, :, 2] = bz[None, :]
    b[:, :, 0] = -0.5 * rc[:, None] * dbz[None, :]
    e = np.zeros((nfr, nfz, 3))
    e[:, :, 0] = e_r * (rc / w.radius)[:, None]
    return with_boris(w, dt=[2.0e-11, 1.0e-7], lifetime=[2.0e-6, 2.0e-4], e_field=e, b_field=b)


def with_primaries(w: Workload, n: int) -> Workload:
    return replace(w, n_primaries=n)
