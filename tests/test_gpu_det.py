"""Deterministic current accumulation (deterministic_j = 1), through the C
ABI.

* The step still matches the oracle to the FP64 tolerances (bit-exact ids,
  cells, positions and momenta; J, E, B within 1e-12 relative): the exact
  integer split of every contribution loses less than 2^-17 of an FP64
  rounding of the largest possible contribution.
* Two runs of the same input, in separate contexts, give the same J, E, B
  and particles bit for bit after several re-sorts, in both precisions and
  with particles on the far-mover path (FP64 atomics give no such
  guarantee).
* A supercell with more particles than the integer LDS sums allow is
  rejected with PIC_ECAPACITY (forced from the host: the kernel returns early
  and sets the error word).
"""
import numpy as np
import pytest

from paper_1608_01009_amd import pic
from paper_1608_01009_amd import workloads as W

from gpu_parity_util import log, one_step_parity

pytestmark = pytest.mark.gpu


def test_det_parity_with_oracle_config1():
    reps, sim = one_step_parity(W.config1(), [0, 19, 20], sim_kwargs=dict(deterministic_j=True))
    for k, rep in reps:
        for key, v in rep.items():
            if key.endswith(".exact"):
                assert v == 1.0, (k, key, v)
    sim.close()


def test_det_parity_thermal_noise_and_shapes():
    one_step_parity(W.scaled(2, (16, 16, 16), 30, seed=71), [0, 7],
                    sim_kwargs=dict(deterministic_j=True))[1].close()
    wl = W.plasma("det-S2h2", (8, 8, 8), 9, 0.05, seed=72, noise=1e-3, S=2, R=7)
    one_step_parity(wl, [0, 6], sim_kwargs=dict(deterministic_j=True, halo=2))[1].close()


def _beam_workload(seed):
    wl = W.scaled(2, (16, 16, 16), 12, seed=seed)
    sp = wl.species[0]
    rng = np.random.default_rng(seed + 1)
    k = sp.n // 8
    sp.ux[:k] = 3.0 + rng.random(k)           # a relativistic fraction leaves the halo
    return wl


def _run(wl, steps, **kw):
    sim = pic.Simulation.from_workload(wl, deterministic_j=True, **kw)
    sim.step(steps)
    F = sim.fields()
    P = sim.particles(0)
    nfar = int(sim.counters()[0])
    sim.close()
    return F, P, nfar


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_det_runs_are_bit_reproducible(precision):
    wl = _beam_workload(73)
    F1, P1, nfar1 = _run(wl, 45, precision=precision)
    F2, P2, nfar2 = _run(wl, 45, precision=precision)
    assert nfar1 > 0 and nfar1 == nfar2
    for c in range(9):
        assert np.array_equal(F1[c], F2[c]), c
    n = P1["n"]
    for key in ("x", "y", "z", "ux", "uy", "uz", "id"):
        assert np.array_equal(P1[key][:n], P2[key][:n]), key
    log(f"  {precision}: 45 steps, {nfar1} far movers, J/E/B and particles bit-identical")


def test_det_matches_atomic_mode_to_rounding():
    wl = W.scaled(2, (16, 16, 16), 20, seed=74)
    out = {}
    for det in (False, True):
        sim = pic.Simulation.from_workload(wl, deterministic_j=det)
        sim.step(1)
        out[det] = sim.fields()
        sim.close()
    for c in range(6, 9):
        a, b = out[False][c], out[True][c]
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


def test_det_rejects_overfull_supercell():
    rng = np.random.default_rng(75)
    N = 20000                                      # all in one supercell of 4^3 cells
    x, y, z = rng.random((3, N)) * 4.0
    u = rng.normal(0, 0.01, (3, N))
    sim = pic.Simulation((8, 8, 8), (1.0, 1.0, 1.0), W.courant_dt(), [(-1.0, 1.0, 0.01, N)],
                         supercell=4, deterministic_j=True)
    try:
        sim.load_particles(0, x, y, z, u[0], u[1], u[2])
        with pytest.raises(pic.PicError) as ei:
            sim.step(1)
        assert ei.value.code == pic.PIC_ECAPACITY
        assert "16383" in ei.value.message
    finally:
        sim.close()
