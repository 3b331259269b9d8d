"""Pins of the oracle's Boris mover (Sec. 3.1 "Boris mover"; vector fields from arrays,
Sec. 3.8 "Vector field").

The push is pinned against closed forms of the discrete map itself:
* uniform B, no E: each push turns v_perp by 2 atan(qB dt / 2m) about B (sense of the Lorentz
  force), v_par and |v| stay; the positions are x_0 + dt * sum of the velocities after each
  push, a geometric series;
* uniform E_z, no B: each push adds qE dt/m to v_z; the positions follow the sum;
* the field lookup: (E_r, E_phi, E_z) of the particle's (r, z) bin turned to Cartesian
  components at its azimuth, zero outside the binning.
Transport with the mover: crossings and time per segment of a beam, transmission through an
absorbing field exp(-mu v dt (K - n_z)) (K pushes to the end, of which the n_z face-crossing
pushes stop the movement without an interaction), the exit energy of a beam accelerated by E_z,
and the energy balance with the field work in the ledger."""
import math

import numpy as np
import pytest

from paper_2503_10263_amd import workloads as W


@pytest.fixture(scope="module")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


def _vacuum(energy=10.0, n_z=10, length=1.0, radius=0.05, species=None, n_primaries=10,
            direction=(0.0, 0.0, 1.0)):
    return W.beam_problem(energy, [], np.zeros(n_z), length, radius=radius,
                          n_primaries=n_primaries, species=species, beam_dir=direction)


def test_rotation_in_uniform_b(oracle_lib):
    b0, dt, n = 0.1, 2.0e-12, 777
    w = W.with_boris(_vacuum(), dt=[dt, 1e-9], lifetime=[1e-5, 1.0],
                     b_field=W.uniform_vector_field(1, 1, (0.0, 0.0, b0)))
    vperp, vpar = 1.3e6, 0.4e6
    x0 = np.array([0.001, 0.002, 0.3])
    out = oracle_lib.boris(w, 0, x0, (vperp, 0.0, vpar), n)
    h = 0.5 * dt * (-W.QE) / W.M_E                     # q dt / 2m of the electron
    phi = 2.0 * math.atan(h * b0)                      # signed turn per push
    # Lorentz force q v x B: v_perp turns by -phi per push in the (x, y) plane (complex form)
    k = np.arange(1, n + 1)
    vk = vperp * np.exp(-1j * phi * k)
    assert abs(out[3] + 1j * out[4] - vk[-1]) < 1e-9 * vperp
    assert abs(out[5] - vpar) < 1e-12 * vpar
    xy = (x0[0] + 1j * x0[1]) + dt * vk.sum()
    assert abs(out[0] + 1j * out[1] - xy) < 1e-9 * vperp * dt * n
    assert abs(out[2] - (x0[2] + n * dt * vpar)) < 1e-12                 # rounding of |z| ~ 0.3 m


def test_acceleration_in_uniform_ez(oracle_lib):
    e0, dt, n = 2.0e3, 1.0e-11, 500
    w = W.with_boris(_vacuum(), dt=[dt, 1e-9], lifetime=[1e-5, 1.0],
                     e_field=W.uniform_vector_field(1, 1, (0.0, 0.0, e0)))
    v0 = np.array([1.0e5, -2.0e5, 3.0e5])
    x0 = np.array([0.0, 0.0, 0.1])
    out = oracle_lib.boris(w, 0, x0, v0, n)
    a = -W.QE * e0 / W.M_E                             # acceleration along z
    k = np.arange(1, n + 1)
    vz = v0[2] + k * a * dt
    assert abs(out[5] - vz[-1]) < 1e-11 * abs(vz[-1])
    assert abs(out[3] - v0[0]) < 1e-9 and abs(out[4] - v0[1]) < 1e-9
    assert abs(out[2] - (x0[2] + dt * vz.sum())) < 1e-11 * abs(dt * vz.sum())
    assert abs(out[0] - n * dt * v0[0]) < 1e-12


def test_field_lookup_cylindrical_bins(oracle_lib):
    """One push with E only: delta v = (q dt / m) E_cart of the bin at the particle's azimuth."""
    nr, nz, R, L, dt = 3, 4, 0.06, 1.2, 1.0e-12
    rng = np.random.default_rng(5)
    ef = rng.normal(size=(nr, nz, 3)) * 1e3
    w = W.with_boris(_vacuum(radius=R, length=L), dt=[dt, 1e-9], lifetime=[1e-5, 1.0],
                     e_field=ef, field_radius=R, field_length=L)          # B: bz = 0
    qdt_m = -W.QE * dt / W.M_E
    for (r, ph, z) in [(0.01, 0.3, 0.1), (0.03, 2.0, 0.5), (0.055, -1.2, 1.1), (0.0, 0.0, 0.7)]:
        x = (r * math.cos(ph), r * math.sin(ph), z)
        out = oracle_lib.boris(w, 0, x, (0.0, 0.0, 0.0), 1)
        ir, iz = min(int(r / R * nr), nr - 1), min(int(z / L * nz), nz - 1)
        er, ep, ez = ef[ir, iz]
        c, s = (math.cos(ph), math.sin(ph)) if r > 0 else (1.0, 0.0)
        expect = qdt_m * np.array([er * c - ep * s, er * s + ep * c, ez])
        np.testing.assert_allclose(out[3:], expect, rtol=1e-12, atol=1e-12 * np.abs(expect).max())
    # outside the binning: no field
    w2 = W.with_boris(_vacuum(radius=R, length=L), dt=[dt, 1e-9], lifetime=[1e-5, 1.0],
                      e_field=ef, field_radius=R / 2, field_length=L / 2)
    out = oracle_lib.boris(w2, 0, (0.04, 0.0, 0.1), (0.0, 0.0, 0.0), 1)
    assert np.all(out[3:] == 0.0)
    out = oracle_lib.boris(w2, 0, (0.01, 0.0, 0.9), (0.0, 0.0, 0.0), 1)
    assert np.all(out[3:] == 0.0)


def test_beam_crossings_and_segment_times(oracle_lib):
    n_z, L, N = 10, 1.0, 200
    E = 10.0
    v = math.sqrt(2.0 * E * W.QE / W.M_E)
    dt = L / (v * 1234.37)                              # 1234.37 pushes per length
    w = W.with_boris(_vacuum(energy=E, n_z=n_z, length=L, n_primaries=N), dt=[dt, 1e-9],
                     lifetime=[1e-5, 1.0], b_field=W.uniform_vector_field(1, 1, (0.0, 0.0, 0.5)))
    t = oracle_lib.run(w)
    K = math.ceil(L / (v * dt))
    c = t["counters"]
    assert c[oracle_lib.C_STEP] == N * K
    assert c[oracle_lib.C_DEATH + W.REASONS.index("exit_high")] == N
    np.testing.assert_array_equal(t["jz"][0, 0, 1:, 1], N)         # every face once, upwards
    cell = t["density_time"][0, 0] / N
    assert abs(cell.sum() - K * dt) < 1e-12 * K * dt
    assert np.all(np.abs(cell - L / n_z / v) <= dt * (1 + 1e-9))


def test_transmission_through_absorbing_field(oracle_lib):
    n_z, L, N, sig, n3 = 40, 1.0, 20000, 1.0e-18, 8.0e17
    E = 5.0
    v = math.sqrt(2.0 * E * W.QE / W.M_E)
    dt = L / (v * 300.45)
    species = [W.electron(e_cut=0.0, edges=np.linspace(0, 10, 11)), W.ion_species("H2+", W.M_H2P, n_bins=10)]
    species[1].edges = np.linspace(0, 10, 11)
    procs = [W.Process(W.RECOMBINATION, W.ELECTRON, W.TARGET_FIELD, 0.0, np.full(256, sig), "rec", partner=1)]
    w = W.beam_problem(E, procs, np.zeros(n_z), L, radius=0.05, n_primaries=N, species=species,
                       n_ion=np.full(n_z, n3))
    w = W.with_boris(w, dt=[dt, 1e-9], lifetime=[1e-5, 1.0])
    t = oracle_lib.run(w)
    K = math.ceil(L / (v * dt))
    mu = n3 * sig
    p = math.exp(-mu * v * dt * (K - n_z))
    trans = t["counters"][oracle_lib.C_DEATH + W.REASONS.index("exit_high")]
    assert abs(trans - N * p) < 4.5 * math.sqrt(N * p * (1 - p)), (trans, N * p)
    # the same count with every push able to interact would be N exp(-mu L): distinguishable
    p_all = math.exp(-mu * v * dt * (K - 1))
    assert abs(N * p - N * p_all) > 3.0 * math.sqrt(N * p * (1 - p))


def test_acceleration_exit_energy_and_field_work(oracle_lib):
    n_z, L, N, e_z = 6, 0.5, 50, -40.0                  # pulls electrons to +z
    E0 = 2.0
    v0 = math.sqrt(2.0 * E0 * W.QE / W.M_E)
    dt = 2.0e-11
    w = W.with_boris(_vacuum(energy=E0, n_z=n_z, length=L, n_primaries=N), dt=[dt, 1e-9],
                     lifetime=[1e-5, 1.0], e_field=W.uniform_vector_field(1, 1, (0.0, 0.0, e_z)))
    w.dens_edges = (np.linspace(0.0, 30.0, 16), np.linspace(0.0, 1.0, 16))
    t = oracle_lib.run(w, hist=True)
    a = -W.QE * e_z / W.M_E
    # discrete kinematics: v_k = v0 + k a dt, z_k = dt * sum v_j; exit at the first z_k >= L
    k = 0
    z = 0.0
    while z < L:
        k += 1
        z += dt * (v0 + k * a * dt)
    e_exit = 0.5 * W.M_E * (v0 + k * a * dt) ** 2 / W.QE
    L_ = t["ledger"]
    got = L_[oracle_lib.L_E_DEATH + W.REASONS.index("exit_high")] / N
    assert abs(got / e_exit - 1.0) < 1e-9
    assert abs(e_exit - (E0 + W.QE * abs(e_z) * L / W.QE)) < abs(e_z) * v0 * dt * 10 + 1.0
    # energy balance: primaries plus field work equal what leaves
    out = L_[oracle_lib.L_E_DEATH:oracle_lib.L_E_DEATH + 2 * oracle_lib.NREASON].sum() + \
        L_[oracle_lib.L_E_EXC] + L_[oracle_lib.L_E_BIND] + L_[oracle_lib.L_E_GAS]
    assert abs(out / (L_[oracle_lib.L_E_PRIMARY] + L_[oracle_lib.L_E_FIELD]) - 1.0) < 1e-12
    h = t["hist"]
    assert np.max(np.abs(h[:, 0] - h[:, 1]) / h[:, 0]) < 1e-11
    # energy bins stop the movement; the bins still add up to the time per segment
    np.testing.assert_allclose(t["density_time_e"].sum(axis=3), t["density_time"], rtol=1e-12)
    assert np.count_nonzero(t["density_time_e"][0].sum(axis=(0, 1))) > 5


def test_boris_descriptor_rules(oracle_lib):
    w = _vacuum()
    w.e_field = W.uniform_vector_field(1, 1, (0.0, 0.0, 1.0))    # E with the drift mover
    w.field_radius, w.field_length = w.radius, w.length
    with pytest.raises(ValueError):
        oracle_lib.run(w)
    w = W.with_boris(_vacuum(), dt=[1e-12, 1e-9], lifetime=[math.inf, 1.0])
    with pytest.raises(ValueError):
        oracle_lib.run(w)
    w = W.with_boris(_vacuum(), dt=[1e-12, 1e-9], lifetime=[1.0, 1.0])   # 1e12 pushes
    with pytest.raises(ValueError):
        oracle_lib.run(w)
