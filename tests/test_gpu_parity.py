"""GPU <-> oracle parity of the whole step, through the C ABI.

One step from an identical state (see gpu_parity_util): bit-exact ids and
cells, x within 2 ulp, u/J/E/B within 1e-12 relative (max norm per array).
Sizes span several supercells and a ragged tail; cases cover the rebin step,
several species, single-supercell (self-overlapping) grids, other supercell
and halo sizes, anisotropic cells, far movers, empty and clustered inputs.
"""
import math

import numpy as np
import pytest

from paper_1608_01009_amd import pic
from paper_1608_01009_amd import workloads as W

from gpu_parity_util import (KEYS, compare, dense_beam_workload, log, one_step_parity,
                             oracle_for, read_state)

pytestmark = pytest.mark.gpu


def test_config1_full_size_steps_0_1_19_20_99():
    wl = W.config1()
    reps, sim = one_step_parity(wl, [0, 1, 19, 20, 99])
    # push bit for bit: the same formula order on both sides
    for k, rep in reps:
        for key, v in rep.items():
            if key.endswith(".exact"):
                assert v == 1.0, (k, key, v)
    sim.close()


def test_thermal_noise_recipe_at_16cubed():
    # the 64^3 / 50 ppc / v_th 0.05 / 1e-3 noise recipe on a 16^3 grid
    wl = W.scaled(2, (16, 16, 16), 50, seed=21)
    reps, sim = one_step_parity(wl, [0, 5, 19, 20])
    sim.close()


def test_two_species_and_ragged_counts():
    base = W.scaled(2, (8, 8, 16), 7, seed=22)
    ions = W.scaled(2, (8, 8, 16), 3, seed=23)
    sp_i = ions.species[0]
    sp_i.charge, sp_i.mass = 1.0, 1836.0
    sp_i.ux *= 0.02
    sp_i.uy *= 0.02
    sp_i.uz *= 0.02
    # drop a ragged number of particles from both
    for sp, keep in ((base.species[0], 7 * 1024 - 13), (sp_i, 3 * 1024 - 101)):
        for k in ("x", "y", "z", "ux", "uy", "uz"):
            setattr(sp, k, np.ascontiguousarray(getattr(sp, k)[:keep]))
    base.species.append(sp_i)
    one_step_parity(base, [0, 3, 19])[1].close()


@pytest.mark.parametrize("n,S,h", [((4, 4, 4), 4, 1), ((4, 8, 12), 4, 1), ((8, 8, 8), 2, 2),
                                   ((6, 6, 6), 1, 1), ((12, 6, 6), 6, 1), ((10, 5, 5), 5, 1),
                                   ((16, 8, 8), 4, 2)])
def test_supercell_and_halo_shapes(n, S, h):
    wl = W.plasma(f"shape-{n}-S{S}-h{h}", n, 9, 0.05, seed=30 + S, noise=1e-3, S=S, R=7)
    one_step_parity(wl, [0, 6, 7], sim_kwargs=dict(halo=h))[1].close()


def test_anisotropic_cells():
    dx = (1.0, 0.5, 2.0)
    wl = W.plasma("aniso", (8, 16, 4), 6, 0.05, seed=40, noise=1e-3, dx=dx,
                  dt=W.courant_dt(dx, 0.9))
    one_step_parity(wl, [0, 1, 4])[1].close()


def test_far_movers_take_the_global_path():
    # a relativistic beam drifts more than the halo before the next re-sort
    wl = W.plasma("beam", (16, 16, 16), 2, 0.0, seed=50, noise=1e-2, R=40)
    sp = wl.species[0]
    rng = np.random.default_rng(51)
    sp.ux[:] = 4.0 + rng.random(sp.n)
    sp.uy[:] = -3.0
    sp.uz[:] = 2.0 * rng.standard_normal(sp.n)
    seen = {}

    def check(sim, k, rep):
        seen[k] = int(sim.counters()[0])

    reps, sim = one_step_parity(wl, [0, 3, 8, 15, 30], extra_check=check)
    assert seen[30] > 0, seen       # the far-mover path was exercised
    sim.close()


def test_empty_species_and_clustered_supercells():
    n = (8, 8, 8)
    rng = np.random.default_rng(60)
    # all particles inside two supercells, the others empty
    N = 1500
    x = rng.random(N) * 4.0
    y = rng.random(N) * 4.0
    z = 4.0 + rng.random(N) * 4.0
    x[::2] += 4.0
    u = rng.normal(0, 0.1, (N, 3))
    fields = [rng.uniform(-1e-2, 1e-2, 512) for _ in range(6)]
    wl = W.Workload("clustered", n, (1.0, 1.0, 1.0), W.courant_dt(), 4, 20, 10,
                    [W.Species(-1.0, 1.0, 0.05, x, y, z, u[:, 0].copy(), u[:, 1].copy(),
                               u[:, 2].copy()),
                     W.Species(1.0, 1836.0, 0.05, np.zeros(0), np.zeros(0), np.zeros(0),
                               np.zeros(0), np.zeros(0), np.zeros(0))],
                    fields)
    one_step_parity(wl, [0, 2])[1].close()


def test_fields_only_vacuum_step():
    n = (8, 6, 10)
    rng = np.random.default_rng(61)
    fields = [rng.standard_normal(480) for _ in range(6)]
    z0 = np.zeros(0)
    wl = W.Workload("vacuum", n, (1.0, 1.0, 1.0), W.courant_dt(), 2, 20, 5,
                    [W.Species(-1.0, 1.0, 0.1, z0, z0, z0, z0, z0, z0)], fields)
    one_step_parity(wl, [0, 1, 3])[1].close()


@pytest.mark.parametrize("n,ppc", [((16, 16, 16), 64), ((8, 8, 8), 200), ((8, 8, 8), 300)])
def test_dense_supercells_staged_resort(n, ppc):
    # 4,096, 12,800 and 19,200 particles per 4^3 supercell: the re-sort order
    # is applied by the LDS-staged permutation (the larger cases overflow its
    # 4,096-value buffer, and the buffers of the neighbourhood re-sort for
    # 4,096 incoming particles and 16,384 classified ones); steps 19 (ends
    # with the re-sort), 20 (the push after it, in stored order) and 21
    wl = W.scaled(2, n, ppc, seed=70 + ppc)
    one_step_parity(wl, [19, 20, 21])[1].close()


def test_resort_with_particles_beyond_the_neighbouring_supercells():
    # every 16th particle (all in odd x cells: the recipe places 2 per cell in
    # x-fastest order) starts at about 0.99 c along x and moves about 2.9
    # cells before the first re-sort, most crossing more than one 2-cell
    # supercell:
    # such a re-sort cannot take the per-supercell (neighbourhood) path and
    # falls back to the global radix sort; the order after it (step 10) and
    # after the next one (step 20) is checked against the oracle
    wl = W.plasma("beam-resort", (32, 16, 16), 2, 0.02, seed=52, noise=1e-2, S=2, R=10)
    sp = wl.species[0]
    rng = np.random.default_rng(53)
    sp.ux[3::16] = 6.0 + rng.random(len(sp.ux[3::16]))
    # the case is what it claims: some particle's supercell moves by more
    # than one between the load and the first re-sort
    sim = pic.Simulation.from_workload(wl)
    a = sim.particles(0)
    sim.step(10)
    b = sim.particles(0)
    sim.close()
    ia, ib = np.argsort(a["id"][:a["n"]]), np.argsort(b["id"][:b["n"]])
    moved = 0
    for key, ns in (("x", 16), ("y", 8), ("z", 8)):
        d = (np.floor(b[key][ib] / 2.0) - np.floor(a[key][ia] / 2.0)) % ns
        moved += int(np.sum((d > 1) & (d < ns - 1)))
    log(f"  particles beyond the neighbouring supercells at the first re-sort: {moved}")
    assert moved > 0
    one_step_parity(wl, [9, 10, 19, 20])[1].close()


def test_dense_resort_with_particles_beyond_the_neighbouring_supercells():
    # the neighbourhood re-sort's queued kernels do nothing (the count of
    # distant particles is not zero), the global sort takes over, and the push
    # after it starts with the staged permutation of that order; steps 19 (ends
    # with the re-sort), 20 and 21 against the oracle
    wl = dense_beam_workload()
    sim = pic.Simulation.from_workload(wl)
    a = sim.particles(0)
    sim.step(20)
    b = sim.particles(0)
    sim.close()
    ia, ib = np.argsort(a["id"][:a["n"]]), np.argsort(b["id"][:b["n"]])
    d = (np.floor(b["x"][ib] / 4.0) - np.floor(a["x"][ia] / 4.0)) % 4
    moved = int(np.sum(d == 2))
    log(f"  dense: particles two supercells on at the first re-sort: {moved}")
    assert moved > 0
    one_step_parity(wl, [19, 20, 21])[1].close()


def test_two_dense_species_resort():
    # electrons and ions, 6,400 of each per 4^3 supercell: both are moved by
    # their re-sort (neighbourhood order, staged permutation) and the step
    # after it pushes both species over one tile load per supercell
    base = W.scaled(2, (8, 8, 8), 100, seed=80)
    ions = W.scaled(2, (8, 8, 8), 100, seed=81)
    sp_i = ions.species[0]
    sp_i.charge, sp_i.mass = 1.0, 1836.0
    sp_i.ux *= 0.02
    sp_i.uy *= 0.02
    sp_i.uz *= 0.02
    base.species.append(sp_i)
    one_step_parity(base, [19, 20, 21])[1].close()
