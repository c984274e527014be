"""Pins of the oracle's laser-plasma extensions: absorbing x boundaries
(first-order Mur on the tangential E, particle removal at the x planes) and
the soft current-sheet laser source.  Each is pinned against physics the
forward scheme must reproduce, not against itself:

* a plane pulse leaving through either x boundary is absorbed (the energy
  left in the box falls below 1 % of what stays in a periodic box);
* the laser sheet radiates a plane wave of amplitude E0 (within 3 %) that
  travels away from the sheet with B_z = E_y, and its envelope arrives at a
  probe plane at the time the distance over c gives;
* particles leaving through x are removed; the Gauss residual at the inside
  nodes and the charge bookkeeping hold to rounding through the removals;
* interpolation next to the boundary uses zero outside the box (brute force
  on a zero-padded lattice), and the source field is E0 sin^2(pi t/T) sin(w t).
"""
import math

import numpy as np


def _grid(orc, n, dt=0.5, S=1):
    return orc.make_grid(n, (1.0, 1.0, 1.0), dt, S, absorb_x=True)


def _pulse(n, x0, width, direction):
    """Plane E_y / B_z pulse travelling along +x (direction 1) or -x (-1)."""
    nx, ny, nz = n
    xe = np.arange(nx, dtype=np.float64)            # E_y at node planes
    xb = xe + 0.5                                   # B_z at half planes
    f = lambda x: np.exp(-((x - x0) / width) ** 2) * np.cos(2 * math.pi * (x - x0) / 12.0)
    Ey = np.tile(f(xe), ny * nz)
    Bz = direction * np.tile(f(xb), ny * nz)
    Bz.reshape(nz, ny, nx)[:, :, nx - 1] = 0.0      # outside slot
    return Ey, Bz


def _run_fields(orc, g, F, steps):
    nc = len(F[0])
    J = [np.zeros(nc) for _ in range(3)]
    for _ in range(steps):
        orc.fdtd(g, F[0:3], F[3:6], J)


def test_mur_absorbs_plane_pulses_at_both_ends(orc):
    n = (240, 2, 2)
    nc = 240 * 4
    for direction, x0 in ((1, 150.0), (-1, 90.0)):
        Ey, Bz = _pulse(n, x0, 10.0, direction)
        F = [np.zeros(nc), Ey.copy(), np.zeros(nc), np.zeros(nc), np.zeros(nc), Bz.copy()]
        Fp = [a.copy() for a in F]
        e0 = sum(float(np.dot(a, a)) for a in F)
        steps = 400                                  # 200 light-cells: the pulse has left
        _run_fields(orc, _grid(orc, n), F, steps)
        gp = orc.make_grid(n, (1.0, 1.0, 1.0), 0.5, 1)
        _run_fields(orc, gp, Fp, steps)
        e_abs = sum(float(np.dot(a, a)) for a in F)
        e_per = sum(float(np.dot(a, a)) for a in Fp)
        assert e_per > 0.9 * e0                      # the periodic box keeps it
        assert e_abs < 0.01 * e0, (direction, e_abs / e0)
        # outside slots held at zero
        for c in (0, 4, 5):
            assert np.all(F[c].reshape(2, 2, 240)[:, :, 239] == 0.0)


def test_laser_sheet_radiates_plane_wave_of_amplitude_e0(orc):
    n = (200, 2, 2)
    nc = 800
    dt = 0.5
    g = _grid(orc, n, dt)
    E0, om, T, plane = 0.19635, 2 * math.pi / 32, 200 * dt, 4
    F = [np.zeros(nc) for _ in range(6)]
    J = [np.zeros(nc) for _ in range(3)]
    probe = 100
    ey, bz = [], []
    for step in range(700):
        for a in J:
            a[:] = 0.0
        orc.add_laser(g, J[1], plane, E0, om, T, (step + 0.5) * dt)
        orc.fdtd(g, F[0:3], F[3:6], J)
        Ey = F[1].reshape(2, 2, 200)[0, 0]
        Bz = F[5].reshape(2, 2, 200)[0, 0]
        ey.append(Ey[probe])
        bz.append(0.5 * (Bz[probe - 1] + Bz[probe]))   # B_z at the E_y plane
    ey, bz = np.array(ey), np.array(bz)
    assert abs(np.max(np.abs(ey)) - E0) <= 0.03 * E0, np.max(np.abs(ey))
    # forward wave: B_z = E_y
    assert np.max(np.abs(bz - ey)) <= 0.03 * E0
    # the envelope peak passes the probe (96 cells downstream) 96 time units
    # after it leaves the sheet (t = T/2)
    env = np.abs(ey)
    t_peak = (np.argmax(env) + 1) * dt
    assert abs(t_peak - (T / 2 + (probe - plane))) <= 16.0
    # nothing is left once the pulse has passed through the far boundary
    e_end = sum(float(np.dot(a, a)) for a in F)
    assert e_end < 1e-3 * E0 ** 2 * 100 * 4
    # the laser field formula
    for t in (0.0, 13.7, 50.0, 99.9, 100.0):
        want = E0 * math.sin(math.pi * t / T) ** 2 * math.sin(om * t)
        assert abs(orc.laser_field(E0, om, T, t) - want) <= 1e-16
    assert orc.laser_field(E0, om, T, -0.1) == 0.0
    assert orc.laser_field(E0, om, T, T + 0.1) == 0.0


def test_particle_removal_keeps_gauss_and_charge_books(orc):
    rng = np.random.default_rng(4)
    n = (16, 8, 8)
    nc = 16 * 64
    sim = orc.OracleSim(n, (1.0, 1.0, 1.0), 0.5, [(-1.0, 1.0, 0.05), (1.0, 1836.0, 0.05)],
                        S=4, R=5, absorb_x=True)
    npart = 400
    x = np.concatenate([rng.uniform(0.0, 2.0, npart // 2), rng.uniform(13.0, 15.0 - 1e-9, npart // 2)])
    ux = np.concatenate([rng.uniform(-3.0, 0.5, npart // 2), rng.uniform(-0.5, 3.0, npart // 2)])
    y, z = rng.uniform(0, 8, npart), rng.uniform(0, 8, npart)
    uy, uz = rng.normal(scale=0.5, size=npart), rng.normal(scale=0.5, size=npart)
    sim.load_particles(0, x, y, z, ux, uy, uz)
    sim.load_particles(1, x.copy(), y.copy(), z.copy(), np.zeros(npart), np.zeros(npart),
                       np.zeros(npart))
    sim.set_fields([rng.normal(scale=1e-3, size=nc) for _ in range(6)])
    F0 = sim.F
    for c in (0, 4, 5):
        F0[c].reshape(8, 8, 16)[:, :, 15] = 0.0
    g0 = sim.gauss().reshape(8, 8, 16)[:, :, 1:15].copy()
    q0 = sim.total_charge()
    removed_seen = 0
    for step in range(12):
        sim.step(1)
        P = sim.particles(0)
        removed_seen = max(removed_seen, int(np.sum(P["x"] < 0)))
        assert np.all((P["x"] == -1.0) | ((P["x"] >= 0.0) & (P["x"] < 15.0)))
        g1 = sim.gauss().reshape(8, 8, 16)[:, :, 1:15]
        assert np.max(np.abs(g1 - g0)) <= 1e-12, step
        # the charge density holds exactly the particles still inside
        assert abs(float(np.sum(sim.rho())) - sim.total_charge()) <= 1e-12
    q1 = sim.total_charge()
    P = sim.particles(0)
    kept = len(P["x"])
    live = int(np.sum(P["x"] >= 0.0))
    assert removed_seen > 50 and kept < npart                 # removal happened and was dropped
    assert abs(q1 - (q0 - (-1.0 * 0.05) * (npart - live))) <= 1e-12
    # since the last re-sort (after step 10) removed particles are marked, not moved
    assert kept - live == int(np.sum(P["x"] == -1.0))


def test_gather_next_to_the_boundary_reads_zero_outside(orc):
    rng = np.random.default_rng(6)
    n = (8, 4, 4)
    nc = 128
    g = _grid(orc, n)
    EB = [rng.normal(size=nc) for _ in range(6)]
    stag = [(0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5), (0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0)]
    for xp in ([0.2, 1.3, 2.7], [0.0, 3.9, 0.1], [6.9, 2.2, 3.3], [6.3, 0.0, 1.0]):
        got = orc.gather(g, EB, xp)
        for c in range(6):
            F = EB[c].reshape(4, 4, 8)
            want = 0.0
            for i in range(-1, 9):
                for j in range(-1, 5):
                    for k in range(-1, 5):
                        wx = max(0.0, 1 - abs(xp[0] - stag[c][0] - i))
                        wy = max(0.0, 1 - abs(xp[1] - stag[c][1] - j))
                        wz = max(0.0, 1 - abs(xp[2] - stag[c][2] - k))
                        if wx * wy * wz == 0.0 or i < 0 or i >= 8:
                            continue
                        want += wx * wy * wz * F[k % 4, j % 4, i]
            assert abs(got[c] - want) <= 1e-14, (xp, c)
