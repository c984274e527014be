"""GPU tests of the C ABI contract: error codes, ownership and device
pointers, call order, long-run invariants and diagnostics against the
oracle, and the full 64^3 / 50 ppc size in the benchmark's configuration."""
import math

import numpy as np
import pytest

import oracle
from paper_1608_01009_amd import pic
from paper_1608_01009_amd import workloads as W

from gpu_parity_util import KEYS, log, max_rel, oracle_for, read_state

pytestmark = pytest.mark.gpu


def _small(n=(8, 8, 8), ppc=4, cap_extra=0):
    wl = W.scaled(1, n, ppc, seed=70)
    sp = wl.species[0]
    sim = pic.Simulation(wl.n, wl.dx, wl.dt, [(sp.charge, sp.mass, sp.weight, sp.n + cap_extra)],
                         supercell=4, rebin_every=20)
    return wl, sim


def test_error_codes():
    wl, sim = _small()
    sp = wl.species[0]
    with pytest.raises(pic.PicError) as e:
        sim.step(1)                                   # before any load
    assert e.value.code == pic.PIC_ESTATE
    x = sp.x.copy()
    x[5] = 8.0                                        # == L: outside [0, L)
    with pytest.raises(pic.PicError) as e:
        sim.load_particles(0, x, sp.y, sp.z, sp.ux, sp.uy, sp.uz)
    assert e.value.code == pic.PIC_EINVAL
    ux = sp.ux.copy()
    ux[3] = np.nan
    with pytest.raises(pic.PicError) as e:
        sim.load_particles(0, sp.x, sp.y, sp.z, ux, sp.uy, sp.uz)
    assert e.value.code == pic.PIC_EINVAL
    big = np.zeros(sp.n + 1)
    with pytest.raises(pic.PicError) as e:
        sim.load_particles(0, big, big, big, big, big, big)
    assert e.value.code == pic.PIC_ECAPACITY
    with pytest.raises(pic.PicError) as e:
        sim.load_particles(3, sp.x, sp.y, sp.z, sp.ux, sp.uy, sp.uz)
    assert e.value.code == pic.PIC_EINVAL
    # a valid load after the failures works
    sim.load_particles(0, *sp.arrays())
    small = {k: np.empty(10) for k in KEYS[:6]}
    small["id"] = np.empty(10, dtype=np.int64)
    with pytest.raises(pic.PicError) as e:
        pic.pic_get_particles(sim.ctx, 0, capacity=10, out=small)
    assert e.value.code == pic.PIC_ECAPACITY
    # non-finite fields make the step report PIC_ENONFINITE
    bad = [np.zeros(512) for _ in range(6)]
    bad[1][100] = np.inf
    sim.set_fields(bad)
    with pytest.raises(pic.PicError) as e:
        sim.step(1)
    assert e.value.code == pic.PIC_ENONFINITE
    sim.close()


def test_load_get_round_trip_and_ids():
    wl, sim = _small()
    sp = wl.species[0]
    ids = np.arange(sp.n, dtype=np.int64)[::-1].copy() * 3 + 7
    sim.load_particles(0, sp.x, sp.y, sp.z, sp.ux, sp.uy, sp.uz, ids)
    got = sim.particles(0)
    o = oracle_for(wl)
    o.load_particles(0, sp.x, sp.y, sp.z, sp.ux, sp.uy, sp.uz, ids)
    want = o.particles(0)
    for k in KEYS:
        assert np.array_equal(got[k], want[k]), k
    sim.close()


def test_device_pointers_and_torch_stream():
    import torch
    dev = torch.device("cuda:0")
    wl = W.scaled(1, (8, 8, 8), 4, seed=71)
    sp = wl.species[0]
    sim = pic.Simulation(wl.n, wl.dx, wl.dt, [(sp.charge, sp.mass, sp.weight, sp.n)],
                         stream="torch")
    t = [torch.from_numpy(a).to(dev) for a in sp.arrays()]
    sim.load_particles(0, *t)
    sim.set_fields([torch.from_numpy(f).to(dev) for f in wl.fields])
    sim.step(3)
    out = {k: torch.empty(sp.n, dtype=torch.float64, device=dev) for k in KEYS[:6]}
    out["id"] = torch.empty(sp.n, dtype=torch.int64, device=dev)
    pic.pic_get_particles(sim.ctx, 0, out=out)
    fo = [torch.empty(512, dtype=torch.float64, device=dev) for _ in range(9)]
    sim.fields(out=fo)
    torch.cuda.synchronize()
    # the same run through host pointers gives the same stored order and state
    sim2 = pic.Simulation.from_workload(wl)
    sim2.step(3)
    host = sim2.particles(0)
    assert np.array_equal(out["id"].cpu().numpy(), host["id"])
    assert np.array_equal(np.floor(out["x"].cpu().numpy()), np.floor(host["x"]))
    assert max_rel(out["ux"].cpu().numpy(), host["ux"]) < 1e-12
    sim.close()
    sim2.close()


def test_long_run_invariants_config1():
    wl = W.config1()
    sim = pic.Simulation.from_workload(wl)
    o = oracle_for(wl)
    o.load_particles(0, *wl.species[0].arrays())
    o.set_fields(wl.fields)
    rho_scale = np.max(np.abs(o.rho()))
    d0 = sim.diagnostics()
    assert d0[4] <= 1e-13 and d0[5] <= 1e-13   # rho re-summed in another atomic order
    for block in range(5):
        sim.step(20)
        d = sim.diagnostics()
        log(f"  diag after {int(d[7])} steps: {d}")
        assert d[4] <= 1e-12 * rho_scale                  # Gauss residual unchanged
        assert d[5] <= 1e-13                              # div B unchanged
        assert d[3] == pytest.approx(-1.0 * 32768 / 8)    # total charge
        assert d[7] == 20 * (block + 1)
    # diagnostics agree with the oracle's on the GPU's state
    F, P = read_state(sim, 1)
    o.set_state([[P[0][k][:P[0]["n"]] for k in KEYS]], F[:6], 0)
    WE, WB = o.field_energy()
    K = o.kinetic()
    assert d[0] == pytest.approx(WE, rel=1e-12)
    assert d[1] == pytest.approx(WB, rel=1e-12, abs=1e-30)
    assert d[2] == pytest.approx(K, rel=1e-10)
    assert sim.counters()[1] == 5                        # re-sorts
    sim.close()


def test_timers_and_counters():
    wl = W.scaled(2, (16, 16, 16), 10, seed=72)
    sim = pic.Simulation.from_workload(wl)
    pic.pic_enable_timers(sim.ctx, True)
    sim.step(25)
    t = pic.pic_get_timers(sim.ctx)
    # one re-sort after step 20: step 21 reads through the re-sort order
    assert t[1] == 24 and t[3] == 1 and t[8] == 25
    assert t[0] > 0 and t[2] > 0 and t[4] > 0 and t[5] > 0 and t[6] > 0
    assert t[7] >= t[0] + t[2] + t[5] and t[9] == 0
    c = sim.counters()
    assert c[1] == 1 and c[2] == 25
    # E/B tile of x-pairs (8 z-planes of 8 rows of 7 pairs, plane pitch padded
    # from 112 to 116 doubles) x 6, padded J tile 3 x 1001, crosser queues
    # 8 waves x 6 x 28 doubles
    assert c[3] == (6 * 116 * 8 + 3 * 1001 + 8 * 6 * 28) * 8
    # mode 2: only the stored-order push+deposit kernel is bracketed
    pic.pic_enable_timers(sim.ctx, 2)
    sim.step(5)
    t = pic.pic_get_timers(sim.ctx)
    assert t[0] > 0 and t[1] == 5 and t[8] == 5
    assert t[2] == 0 and t[4] == 0 and t[5] == 0 and t[6] == 0 and t[7] == 0
    # mode 3: that kernel on the timed steps 0, 7, 14 only (the re-sort after
    # step 40 falls between the samples)
    pic.pic_enable_timers(sim.ctx, 3)
    sim.step(15)
    t = pic.pic_get_timers(sim.ctx)
    assert t[0] > 0 and t[1] == 3 and t[8] == 15
    assert t[2] == 0 and t[4] == 0 and t[5] == 0 and t[6] == 0 and t[7] == 0
    with pytest.raises(pic.PicError) as ei:
        pic.pic_enable_timers(sim.ctx, 4)
    assert ei.value.code == pic.PIC_EINVAL
    sim.close()


def test_long_run_invariants_64cubed_50ppc():
    """The benchmark's workload (13,107,200 particles) through its 200 steps and
    ten re-sorts: after every re-sort period the Gauss residual and div B are
    unchanged to rounding (the deposition conserves charge exactly), the total
    charge is exact, and at the end the field and kinetic energies the library
    reports equal the oracle's evaluation of the GPU's state."""
    wl = W.config2()
    sp = wl.species[0]
    sim = pic.Simulation.from_workload(wl)
    o = oracle_for(wl)
    o.load_particles(0, *sp.arrays())
    o.set_fields(wl.fields)
    rho_scale = np.max(np.abs(o.rho()))
    q = sp.charge * sp.weight * sp.n
    for block in range(10):
        sim.step(wl.R)
        d = sim.diagnostics()
        assert d[4] <= 1e-12 * rho_scale                  # Gauss residual unchanged
        assert d[5] <= 1e-13                              # div B unchanged
        assert d[3] == pytest.approx(q, rel=1e-12)        # total charge
        assert d[7] == wl.R * (block + 1)
    log(f"  64^3 x 50 after {int(d[7])} steps: gauss drift {d[4]:.2e} (rho scale "
        f"{rho_scale:.2e}), div B drift {d[5]:.2e}, W_E {d[0]:.6e} W_B {d[1]:.6e} K {d[2]:.6e}")
    assert sim.counters()[1] == 10                       # re-sorts
    F, P = read_state(sim, 1)
    sim.close()
    o.set_state([[P[0][k][:P[0]["n"]] for k in KEYS]], F[:6], 0)
    del F, P
    WE, WB = o.field_energy()
    assert d[0] == pytest.approx(WE, rel=1e-12)
    assert d[1] == pytest.approx(WB, rel=1e-12)
    assert d[2] == pytest.approx(o.kinetic(), rel=1e-10)


def test_full_size_64cubed_50ppc_one_step():
    """The benchmark's workload at its full size (13,107,200 particles, S = 4,
    h = 1): one step from the loaded state, checked against the oracle's
    full step (all particles, J, E, B)."""
    wl = W.config2()
    log(f"  full size: {wl.nparticles} particles")
    sim = pic.Simulation.from_workload(wl)
    F0, P0 = read_state(sim, 1)
    sim.step(1)
    gF, gP = read_state(sim, 1)
    o = oracle_for(wl)
    o.set_state([[P0[0][k][:P0[0]["n"]] for k in KEYS]], F0[:6], 0)
    log("  oracle step at full size")
    o.step(1)
    from gpu_parity_util import compare
    rep = compare(gF, gP, o, wl.n, tag="64^3x50")
    log(f"  full size parity: {rep}")
    d = sim.diagnostics()
    assert d[4] <= 1e-12 * 50 * 0.02 * 8
    sim.close()
