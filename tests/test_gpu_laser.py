"""GPU tests of the laser-plasma extensions (absorbing x boundaries, particle
removal, laser current sheet) against the oracle.

* one step from an identical state, the protocol and tolerances of the
  periodic parity tests, on a small laser slab (64 x 8 x 8 cells, electrons
  and protons in 24 <= x < 56, wavelength 16 cells, a0 = 1) with a third
  species of relativistic electrons leaving through both x boundaries: at
  the start, around a re-sort that drops removed particles, and while the
  laser pulse crosses the slab; removed particles (x = -1) and the stored
  order agree bit for bit;
* the full-size slab (256 x 128 x 128 cells, 33.6 M particles, the launch
  configuration the benchmark times): one step late in the run, with the pulse
  inside the plasma and ending with a re-sort, against the oracle's step;
* the laser in vacuum: fields after 300 steps against the oracle's;
* the diagnostics (Gauss residual at the inside nodes, charge of the
  particles inside) and the error codes of the boundary and source settings.
"""
import numpy as np
import pytest

import oracle
from gpu_layout import LayoutOracle
from paper_1608_01009_amd import pic
from paper_1608_01009_amd import workloads as W

from gpu_parity_util import KEYS, compare, log, max_rel

pytestmark = pytest.mark.gpu


def _small_slab(seed=21):
    wl = W.laser_slab(n=(64, 8, 8), slab=(24, 56), ppc=2, seed=seed, wavelength=16.0,
                      name="laser-slab-64x8x8")
    rng = np.random.default_rng(seed)
    nb = 512
    x = np.concatenate([rng.uniform(1.0, 4.0, nb // 2), rng.uniform(58.0, 62.9, nb // 2)])
    ux = np.concatenate([rng.uniform(-3.0, -0.5, nb // 2), rng.uniform(0.5, 3.0, nb // 2)])
    beam = W.Species(-1.0, 1.0, 0.01, x, rng.uniform(0, 8, nb), rng.uniform(0, 8, nb), ux,
                     rng.normal(scale=0.3, size=nb), rng.normal(scale=0.3, size=nb))
    wl.species.append(beam)
    return wl


def _oracle(wl, F, P, k):
    o = LayoutOracle(wl.n, wl.dx, wl.dt, [(s.charge, s.mass, s.weight) for s in wl.species],
                         S=wl.S, R=wl.R, absorb_x=True, laser=wl.laser)
    o.set_state([[p[k_][:p["n"]] for k_ in KEYS] for p in P], F[:6], k % wl.R, step_count=k)
    return o


def _state(sim, ns):
    return sim.fields(), [sim.particles(s) for s in range(ns)]


def test_laser_slab_one_step_parity():
    wl = _small_slab()
    ns = len(wl.species)
    sim = pic.Simulation.from_workload(wl)
    at = 0
    removed = 0
    for k in (0, 1, 19, 20, 39, 60, 100, 159, 160):
        if k > at:
            sim.step(k - at)
            at = k
        F0, P0 = _state(sim, ns)
        sim.step(1)
        at += 1
        F1, P1 = _state(sim, ns)
        o = _oracle(wl, F0, P0, k)
        o.step(1)
        log(f"  step {k} -> {k + 1}: counts {[p['n'] for p in P1]}, removed marked "
            f"{[int(np.sum(p['x'][:p['n']] < 0)) for p in P1]}")
        rep = compare(F1, P1, o, wl.n, tag=f"slab step {k}")
        removed += int(np.sum(P1[2]["x"][:P1[2]["n"]] < 0))
        log(f"    {rep}")
    # particles left through both boundaries and the re-sorts dropped them
    assert sim.particles(2)["n"] < 512
    assert removed > 0
    # the pulse reached the slab: the electrons there moved
    ux = sim.particles(0)["uy"]
    assert np.max(np.abs(ux)) > 0.05
    sim.close()


def test_laser_slab_two_species_one_launch_parity():
    """Electrons (with the leaving beam merged in) and protons: the context
    pushes both species in one launch over one tile load per supercell; the
    one-step protocol as above, removal and re-sorts included.  A cluster of
    slow electrons in the supercells at x = 12..16, next to empty ones at
    x = 8..12 and without protons, gives supercells where one species is
    absent."""
    wl = _small_slab(seed=25)
    beam = wl.species.pop()
    rng = np.random.default_rng(26)
    nc = 40
    cluster = W.Species(-1.0, 1.0, 0.01, rng.uniform(12.5, 15.5, nc), rng.uniform(0, 8, nc),
                        rng.uniform(0, 8, nc), *[rng.normal(scale=0.05, size=nc) for _ in range(3)])
    e = wl.species[0]
    for k in ("x", "y", "z", "ux", "uy", "uz"):
        setattr(e, k, np.concatenate([getattr(e, k), getattr(beam, k), getattr(cluster, k)]))
    sim = pic.Simulation.from_workload(wl)
    at = 0
    for k in (0, 1, 19, 20, 41, 120):
        if k > at:
            sim.step(k - at)
            at = k
        F0, P0 = _state(sim, 2)
        sim.step(1)
        at += 1
        F1, P1 = _state(sim, 2)
        o = _oracle(wl, F0, P0, k)
        o.step(1)
        compare(F1, P1, o, wl.n, tag=f"two-species slab step {k}")
        log(f"  step {k} -> {k + 1}: counts {[p['n'] for p in P1]}")
    assert sim.particles(0)["n"] < e.n                  # beam electrons left and were dropped
    sim.close()


@pytest.mark.parametrize("plane", [1, 18])
def test_laser_sheet_next_to_a_mur_plane_parity(plane):
    """The source sheet on the plane next to a Mur plane (1 or n0 - 2) on a
    box 20 cells wide: the Mur update of the boundary plane recomputes its
    neighbour's new E_y from that plane's J, and on this width some rows of
    the two planes fall into different waves.  The one-step protocol checks
    that the source enters E_y once and the stored J once."""
    wl = W.laser_slab(n=(20, 8, 8), slab=(6, 14), ppc=2, seed=31, wavelength=8.0,
                      envelope_steps=60, plane=plane, name=f"laser-plane-{plane}")
    sim = pic.Simulation.from_workload(wl)
    at = 0
    for k in (0, 5, 19, 20, 33):
        if k > at:
            sim.step(k - at)
            at = k
        F0, P0 = _state(sim, 2)
        sim.step(1)
        at += 1
        F1, P1 = _state(sim, 2)
        o = _oracle(wl, F0, P0, k)
        o.step(1)
        rep = compare(F1, P1, o, wl.n, tag=f"plane {plane} step {k}")
        log(f"  plane {plane} step {k} -> {k + 1}: Ey {rep['Ey']:.2e} Jy {rep['Jy']:.2e}")
    assert np.max(np.abs(sim.fields()[1])) > 0.1 * wl.laser[0]    # the pulse is in the box
    sim.close()


def test_laser_in_vacuum_matches_oracle():
    n = (96, 4, 4)
    wl = W.laser_slab(n=n, slab=(40, 44), ppc=1, wavelength=16.0, name="vacuum")
    for s in wl.species:
        for a in ("x", "y", "z", "ux", "uy", "uz"):
            setattr(s, a, getattr(s, a)[:0].copy())
    sim = pic.Simulation.from_workload(wl)
    sim.step(300)
    F = sim.fields()
    o = LayoutOracle(wl.n, wl.dx, wl.dt, [(s.charge, s.mass, s.weight) for s in wl.species],
                         S=wl.S, R=wl.R, absorb_x=True, laser=wl.laser)
    for s in range(2):
        o.load_particles(s, *[np.zeros(0)] * 6)
    o.set_fields(wl.fields)
    o.step(300)
    worst = 0.0
    for c in range(9):
        worst = max(worst, max_rel(F[c], o.F[c]))
    log(f"  vacuum laser, 300 steps: max rel {worst:.2e}, "
        f"exact {np.mean([np.array_equal(F[c], o.F[c]) for c in range(9)]):.2f}")
    assert worst <= 1e-14
    assert np.max(np.abs(F[1])) > 0.3 * wl.laser[0]      # the pulse is in the box
    sim.close()


def test_diagnostics_and_error_codes():
    wl = _small_slab(seed=23)
    ns = len(wl.species)
    sim = pic.Simulation.from_workload(wl)
    d0 = sim.diagnostics()
    q0 = d0[3]
    sim.step(45)
    d = sim.diagnostics()
    P = [sim.particles(s) for s in range(ns)]
    live = [int(np.sum(p["x"][:p["n"]] >= 0)) for p in P]
    q = sum(s.charge * s.weight * nl for s, nl in zip(wl.species, live))
    assert d[3] == pytest.approx(q, rel=1e-12, abs=1e-12)
    assert q != q0                                       # beam charge left the box
    rho_scale = 2 * wl.meta["n0"]
    assert d[4] <= 1e-12 * rho_scale                     # Gauss at the inside nodes
    assert d[5] <= 1e-13
    # settings
    with pytest.raises(pic.PicError) as e:
        sim.set_laser(0.1, 0.3, 10.0, 0)                 # plane on the boundary
    assert e.value.code == pic.PIC_EINVAL
    with pytest.raises(pic.PicError) as e:
        sim.set_laser(0.1, 0.3, 0.0, 5)                  # duration
    assert e.value.code == pic.PIC_EINVAL
    x = wl.species[0].x.copy()
    x[0] = 63.0                                          # n0 - 1: outside the particle range
    sp = wl.species[0]
    with pytest.raises(pic.PicError) as e:
        sim.load_particles(0, x, sp.y, sp.z, sp.ux, sp.uy, sp.uz)
    assert e.value.code == pic.PIC_EINVAL
    with pytest.raises(pic.PicError) as e:
        sim.record(5)
    assert e.value.code == pic.PIC_EINVAL
    sim.close()
    per = pic.Simulation((8, 8, 8), (1.0, 1.0, 1.0), 0.25, [(-1.0, 1.0, 1.0, 10)])
    with pytest.raises(pic.PicError) as e:
        per.set_laser(0.1, 0.3, 10.0, 3)
    assert e.value.code == pic.PIC_EINVAL
    per.close()


@pytest.mark.timeout(400)
def test_laser_slab_full_size_one_step():
    """The laser-plasma slab at its full size (256 x 128 x 128 cells, 33,554,432
    particles, both species in one launch, re-sorted every 10 steps) in the
    configuration the benchmark times: 509 steps on the GPU (the pulse has
    entered the plasma: electrons at up to 0.8 c, cell crossers and far movers),
    then step 509 -> 510, which ends with a re-sort, against the oracle's step
    from the same state: every particle (stored order bit for bit, cells bit
    for bit, positions within 2 ulp, momenta 1e-12), J, E and B."""
    wl = W.config3()
    k = 509
    sim = pic.Simulation.from_workload(wl)
    log(f"  full-size slab: {wl.nparticles} particles, {k} steps on the GPU")
    sim.step(k)
    F0, P0 = _state(sim, 2)
    sim.step(1)
    F1, P1 = _state(sim, 2)
    log(f"  global-path pushes so far: {int(sim.counters()[0])}")
    sim.close()
    u = P0[0]["uy"][:P0[0]["n"]]
    log(f"  electrons max |u_y| {np.max(np.abs(u)):.2f}")
    assert np.max(np.abs(u)) > 0.3
    o = _oracle(wl, F0, P0, k)
    del F0, P0
    log("  oracle step at full size")
    o.step(1)
    rep = compare(F1, P1, o, wl.n, tag=f"full-size slab step {k}")
    log(f"  {rep}")
