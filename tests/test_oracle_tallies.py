"""Pins of the oracle's geometry and tallies (closed-form flight times and face
crossings), conservation of energy and particles per history, and additivity of the
tallies over disjoint primary ranges."""
import math

import numpy as np
import pytest

from paper_2503_10263_amd import workloads as W


def speed(e_ev, m):
    return math.sqrt(2.0 * e_ev * W.QE / m)


def test_straight_line_cell_times_and_crossings(oracle_lib):
    """No gas: a ray from the axis at polar angle theta crosses r-face k at path r_k/sin(theta)
    and z-face j at path z_j/cos(theta); time per (r,z) cell is the path inside it over v."""
    N, e = 50, 100.0
    R, L, n_r, n_z = 0.04, 0.2, 4, 10
    th = math.radians(20.0)
    d = (math.sin(th), 0.0, math.cos(th))
    w = W.beam_problem(e, [], np.zeros(n_z), L, radius=R, n_r=n_r, n_primaries=N,
                       beam_pos=(0.0, 0.0, 0.0), beam_dir=d)
    t = oracle_lib.run(w)
    v = speed(e, W.M_E)
    events = sorted([(R * k / n_r / math.sin(th), "r", k) for k in range(1, n_r + 1)] +
                    [(L * j / n_z / math.cos(th), "z", j) for j in range(1, n_z + 1)])
    expect = np.zeros((n_r, n_z))
    jr = np.zeros((n_r + 1, n_z, 2), np.int64)
    jz = np.zeros((n_r, n_z + 1, 2), np.int64)
    s0, ir, iz = 0.0, 0, 0
    for s, kind, k in events:
        expect[ir, iz] += (s - s0) / v
        s0 = s
        if kind == "r":
            jr[k, iz, 1] += N
            if k == n_r:
                break
            ir = k
        else:
            jz[ir, k, 1] += N
            if k == n_z:
                break
            iz = k
    np.testing.assert_allclose(t["density_time"][0], N * expect, rtol=1e-12, atol=1e-25)
    np.testing.assert_array_equal(t["jr"][0], jr)
    np.testing.assert_array_equal(t["jz"][0], jz)
    c = t["counters"]
    assert c[oracle_lib.C_DEATH + W.REASONS.index("wall")] == N


def test_guiding_centre_flight_time(oracle_lib):
    """Uniform B, no gas: the particle drifts along z with v*mu, so each z-cell takes
    dz/(v mu); the guiding centre keeps its radius, so no r-face is crossed."""
    N, e = 40, 500.0
    R, L, n_r, n_z = 0.045, 1.0, 8, 16
    mu = 0.6
    d = (math.sqrt(1 - mu**2), 0.0, mu)
    w = W.beam_problem(e, [], np.zeros(n_z), L, radius=R, n_r=n_r, n_primaries=N, bz=2.5,
                       beam_pos=(0.012, 0.0, 0.0), beam_dir=d)
    t = oracle_lib.run(w)
    v = speed(e, W.M_E)
    # guiding centre radius: x + v_y/omega with omega = q B / m
    om = -W.QE * 2.5 / W.M_E
    gx, gy = 0.012 + 0.0, -v * d[0] / om
    ir = int(math.hypot(gx, gy) / (R / n_r))
    got = t["density_time"][0]
    exp_ = np.zeros((n_r, n_z))
    exp_[ir, :] = N * (L / n_z) / (v * mu)
    np.testing.assert_allclose(got, exp_, rtol=1e-12, atol=1e-25)
    assert t["counters"][oracle_lib.C_RCROSS] == 0
    assert t["counters"][oracle_lib.C_DEATH + W.REASONS.index("exit_high")] == N


def test_guiding_centre_wall_at_birth(oracle_lib):
    """An orbit whose guiding-centre radius plus gyro radius reaches R is lost to the wall."""
    e, B = 2000.0, 0.5
    v = speed(e, W.M_E)
    r_l = v * W.M_E / (W.QE * B)
    R = 0.01
    # electron moving along -y: the guiding centre lies r_L further out, at x + v_y/omega
    om = -W.QE * B / W.M_E
    d = np.array([0.0, -1.0, 1e-3])
    d /= np.linalg.norm(d)
    for x0, lost in [(R - 2.2 * r_l, False), (R - 1.5 * r_l, True)]:
        gx = x0 + v * d[1] / om
        w = W.beam_problem(e, [], np.zeros(2), 0.1, radius=R, n_r=4, n_primaries=3, bz=B,
                           beam_pos=(x0, 0.0, 0.05), beam_dir=tuple(d))
        t = oracle_lib.run(w)
        wall = t["counters"][oracle_lib.C_DEATH + W.REASONS.index("wall")]
        assert (abs(gx) + r_l >= R) == lost
        assert wall == (3 if lost else 0)
        if lost:
            assert t["jr"][0, 4].sum() == 3


def _check_conservation(oracle_lib, w, n):
    t = oracle_lib.run(w, 0, n, digests=True, hist=True)
    h = t["hist"][:n]
    np.testing.assert_array_equal(h[:, 2], h[:, 3])          # every particle deleted once
    rel = np.abs(h[:, 0] - h[:, 1]) / h[:, 0]
    assert rel.max() < 1e-11
    c = t["counters"]
    n_ion_proc = sum(c[oracle_lib.C_PROC + i] for i, p in enumerate(w.processes)
                     if p.kind == W.IONIZATION)
    # each ionization makes one electron and one ion (charge conservation)
    assert c[oracle_lib.C_BIRTH] == n + n_ion_proc
    assert c[oracle_lib.C_BIRTH + 1] == n_ion_proc
    nr = oracle_lib.NREASON
    deaths = c[oracle_lib.C_DEATH:oracle_lib.C_DEATH + 2 * nr].reshape(2, nr)
    assert deaths[0].sum() == c[oracle_lib.C_BIRTH] and deaths[1].sum() == c[oracle_lib.C_BIRTH + 1]
    L = t["ledger"]
    total_out = L[oracle_lib.L_E_DEATH:oracle_lib.L_E_DEATH + 2 * nr].sum() + \
        L[oracle_lib.L_E_EXC] + L[oracle_lib.L_E_BIND] + L[oracle_lib.L_E_GAS]
    assert abs(total_out / L[oracle_lib.L_E_PRIMARY] - 1.0) < 1e-12
    # recombination deletions equal the deletions logged in the partner's field
    assert deaths[0, W.REASONS.index("recombined")] == t["recomb"][1].sum()
    assert deaths[1, W.REASONS.index("recombined")] == t["recomb"][0].sum()
    return t


def test_conservation_tiny(oracle_lib):
    _check_conservation(oracle_lib, W.cfg_tiny(n_primaries=3000, column_cm2=1e18), 3000)


def test_conservation_full_capped(oracle_lib):
    w = W.cfg_full(n_primaries=40)
    w.species[W.ION].cap = 2000
    t = _check_conservation(oracle_lib, w, 40)
    c = t["counters"]
    assert c[oracle_lib.C_DEATH + oracle_lib.NREASON + W.REASONS.index("cap")] > 0


def test_gas_at_rest_energy_budget(oracle_lib):
    """T = 0 and no ionization target motion: the ionization frame term vanishes."""
    w = W.cfg_tiny(n_primaries=1000, column_cm2=1e18)
    w.t_gas = 0.0
    t = oracle_lib.run(w, hist=True)
    L = t["ledger"]
    assert L[oracle_lib.L_E_GAS] >= 0.0           # elastic recoil only removes energy
    assert t["counters"][oracle_lib.C_TARGET_REDRAW] == 0


def test_tallies_additive_over_pid_ranges(oracle_lib):
    w = W.cfg_tiny(n_primaries=600, column_cm2=1e17, bz=2.5, n_r=4, n_z=8)
    w.planes = [0, 4, 8]
    full = oracle_lib.run(w, 0, 600, digests=True)
    a = oracle_lib.run(w, 0, 277, digests=True)
    b = oracle_lib.run(w, 277, 600, digests=True)
    for k in ["counters", "recomb", "jz", "jr", "spectra"]:
        np.testing.assert_array_equal(full[k], a[k] + b[k])
    np.testing.assert_array_equal(full["digests"], a["digests"] + b["digests"])
    np.testing.assert_allclose(full["density_time"], a["density_time"] + b["density_time"], rtol=1e-12)


def test_rejects_bad_ranges(oracle_lib):
    w = W.cfg_tiny(n_primaries=10)
    with pytest.raises(ValueError):
        oracle_lib.run(w, 0, 11)
    with pytest.raises(ValueError):
        oracle_lib.run(w, 5, 4)


def test_fields_pencil_beam_closed_form(oracle_lib):
    """eq. (3)-(5): a pencil beam of N primaries at speed v with activity a has density
    a/(v A_ring) in the central ring and current a/A_ring through every z-face it crosses."""
    N, e, act = 200, 50.0, 3.0e7
    R, L, n_r, n_z = 0.04, 0.5, 4, 5
    w = W.beam_problem(e, [], np.zeros(n_z), L, radius=R, n_r=n_r, n_primaries=N)
    t = oracle_lib.run(w)
    f = oracle_lib.fields(w, t, N, act)
    v = speed(e, W.M_E)
    area = math.pi * (R / n_r) ** 2
    np.testing.assert_allclose(f["density"][0, 0], act / (v * area), rtol=1e-12)
    assert np.all(f["density"][0, 1:] == 0.0) and np.all(f["density"][1] == 0.0)
    # the beam starts on face 0 and crosses faces 1..n_z
    assert f["jz"][0, 0, 0] == 0.0
    np.testing.assert_allclose(f["jz"][0, 0, 1:], act / area, rtol=1e-12)
    assert np.all(f["jr"] == 0.0)
