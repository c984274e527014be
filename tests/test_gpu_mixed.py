"""GPU mixed-precision variant (PIC_FP32_MIXED) against the oracle's
mixed-precision loop and against the FP64 oracle, through the C ABI.

One step from an identical state (the GPU's state S_k read back; the oracle
steps from it; compared with the GPU's S_{k+1}):
* ids (the stored order) and positions (cell + FP32 offset) and FP32 momenta:
  bit for bit against the mixed-precision oracle (same FP32 expressions);
* J per node: |J_gpu - J_oracle| <= (n_node + 4) 2^-24 sum_node |contribution|,
  the bound of summing n_node FP32 contributions in another order plus a few
  units of rounding in each contribution (the GPU multiplies by 1/12 where
  the oracle divides by 12);
* E and B: the J bound carried through one Yee update.
Against the FP64 oracle the same step differs by FP32 rounding: positions,
momenta and J within the bounds the oracle pins use; the observed errors are
printed.
"""
import numpy as np
import pytest

from paper_1608_01009_amd import pic
from paper_1608_01009_amd import workloads as W

from gpu_parity_util import KEYS, dense_beam_workload, log, read_state

from gpu_layout import LayoutOracle

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -24


def _mixed_oracle(wl, precision="mixed"):
    o = LayoutOracle(wl.n, wl.dx, wl.dt, [(s.charge, s.mass, s.weight) for s in wl.species],
                         S=wl.S, R=wl.R, precision=precision)
    o.collect_abs = precision == "mixed"
    return o


def _compare_mixed(gF, gP, o, wl, tag):
    for s, gp in enumerate(gP):
        op = o.particles(s)
        n = gp["n"]
        assert n == len(op["x"]), tag
        assert np.array_equal(gp["id"][:n], op["id"]), f"{tag}: order differs"
        for k in ("x", "y", "z", "ux", "uy", "uz"):
            assert np.array_equal(gp[k][:n], op[k]), (
                f"{tag}: {k} differs, max {np.max(np.abs(gp[k][:n] - op[k]))}")
    tolJ = []
    for d in range(3):
        g = gF[6 + d]
        w = o.F[6 + d]
        bound = (o.Jcnt[d] + 4) * EPS32 * o.Jabs[d]
        err = np.abs(g - w)
        assert np.all(err <= bound + 1e-300), (
            f"{tag}: J{'xyz'[d]} max excess {np.max(err - bound)}")
        tolJ.append(np.max(bound))
    dt = wl.dt
    tE = dt * max(tolJ) * 1.01
    for c in range(3):
        scale = np.max(np.abs(o.F[c]))
        assert np.max(np.abs(gF[c] - o.F[c])) <= tE + 1e-12 * scale, f"{tag}: E{'xyz'[c]}"
    tB = 2.0 * dt * tE / min(wl.dx)
    for c in range(3, 6):
        scale = np.max(np.abs(o.F[c]))
        assert np.max(np.abs(gF[c] - o.F[c])) <= tB + 1e-12 * scale, f"{tag}: B{'xyz'[c - 3]}"


def _run(wl, ks, check, sim_kwargs=None):
    sim = pic.Simulation.from_workload(wl, precision="mixed", **(sim_kwargs or {}))
    nsp = len(wl.species)
    cur = 0
    try:
        for k in ks:
            log(f"  mixed {wl.name}: advancing GPU to step {k}")
            if k > cur:
                sim.step(k - cur)
            F, P = read_state(sim, nsp)
            sim.step(1)
            cur = k + 1
            gF, gP = read_state(sim, nsp)
            check(wl, k, F, P, gF, gP)
        return int(sim.counters()[0])
    finally:
        sim.close()


def _against_mixed_oracle(wl, k, F, P, gF, gP):
    o = _mixed_oracle(wl)
    o.set_state([[p[key][:p["n"]] for key in KEYS] for p in P], F[:6], k % wl.R)
    o.step(1)
    _compare_mixed(gF, gP, o, wl, f"{wl.name} k={k}")
    log(f"  mixed {wl.name} k={k}: positions, momenta, ids bit for bit; J, E, B within bounds")


def test_mixed_one_step_bit_exact_against_mixed_oracle():
    _run(W.scaled(2, (16, 16, 16), 20, seed=41), [0, 1, 19, 20], _against_mixed_oracle)


def test_mixed_two_species_ragged():
    base = W.scaled(2, (8, 8, 16), 9, seed=42)
    ions = W.scaled(2, (8, 8, 16), 3, seed=43)
    sp_i = ions.species[0]
    sp_i.charge, sp_i.mass = 1.0, 1836.0
    for k in ("ux", "uy", "uz"):
        setattr(sp_i, k, getattr(sp_i, k) * 0.02)
    for k in ("x", "y", "z", "ux", "uy", "uz"):
        setattr(base.species[0], k, np.ascontiguousarray(getattr(base.species[0], k)[:9 * 1024 - 7]))
    base.species.append(sp_i)
    _run(base, [0, 19], _against_mixed_oracle)


@pytest.mark.parametrize("n,S,h", [((4, 4, 4), 4, 1), ((8, 8, 8), 2, 2), ((6, 6, 6), 1, 1),
                                   ((16, 8, 8), 4, 2)])
def test_mixed_supercell_and_halo_shapes(n, S, h):
    wl = W.plasma(f"mixed-shape-{n}-S{S}-h{h}", n, 9, 0.05, seed=50 + S, noise=1e-3, S=S, R=7)
    _run(wl, [0, 6], _against_mixed_oracle, sim_kwargs=dict(halo=h))


def test_mixed_anisotropic_cells():
    dx = (1.0, 0.5, 2.0)
    wl = W.plasma("mixed-aniso", (8, 16, 4), 6, 0.05, seed=52, noise=1e-3, dx=dx,
                  dt=W.courant_dt(dx, 0.9))
    _run(wl, [0, 3], _against_mixed_oracle)


def test_mixed_far_movers():
    # a relativistic beam drifts more than the halo before the next re-sort
    wl = W.plasma("mixed-beam", (16, 16, 16), 2, 0.0, seed=53, noise=1e-2, R=40)
    sp = wl.species[0]
    rng = np.random.default_rng(54)
    sp.ux[:] = 4.0 + rng.random(sp.n)
    sp.uy[:] = -3.0
    sp.uz[:] = 2.0 * rng.standard_normal(sp.n)
    nfar = _run(wl, [0, 8, 30], _against_mixed_oracle)
    assert nfar > 0


def test_mixed_clustered_and_empty():
    n = (8, 8, 8)
    rng = np.random.default_rng(62)
    N = 1500
    x = rng.random(N) * 4.0
    y = rng.random(N) * 4.0
    z = 4.0 + rng.random(N) * 4.0
    x[::2] += 4.0
    u = rng.normal(0, 0.1, (N, 3))
    fields = [rng.uniform(-1e-2, 1e-2, 512) for _ in range(6)]
    wl = W.Workload("mixed-clustered", n, (1.0, 1.0, 1.0), W.courant_dt(), 4, 20, 10,
                    [W.Species(-1.0, 1.0, 0.05, x, y, z, u[:, 0].copy(), u[:, 1].copy(),
                               u[:, 2].copy()),
                     W.Species(1.0, 1836.0, 0.05, np.zeros(0), np.zeros(0), np.zeros(0),
                               np.zeros(0), np.zeros(0), np.zeros(0))],
                    fields)
    _run(wl, [0, 2], _against_mixed_oracle)


def test_mixed_against_fp64_oracle_error_statement():
    wl = W.scaled(2, (16, 16, 16), 20, seed=44)
    errs = {}

    def check(wl, k, F, P, gF, gP):
        o = _mixed_oracle(wl, precision="fp64")
        o.set_state([[p[key][:p["n"]] for key in KEYS] for p in P], F[:6], k % wl.R)
        o.step(1)
        om = _mixed_oracle(wl)               # for the per-node J bounds
        om.set_state([[p[key][:p["n"]] for key in KEYS] for p in P], F[:6], k % wl.R)
        om.step(1)
        gp, op = gP[0], o.particles(0)
        n = gp["n"]
        assert np.array_equal(gp["id"][:n], op["id"])
        umax = max(np.max(np.abs(op[k])) for k in ("ux", "uy", "uz"))
        sp = wl.species[0]
        h = abs(sp.charge * wl.dt / (2 * sp.mass))
        emax = max(np.max(np.abs(f)) for f in F[:3])
        for d, key in enumerate(("x", "y", "z")):
            dx = np.abs(gp[key][:n] - op[key])
            dx = np.minimum(dx, wl.n[d] - dx)
            errs[key] = float(dx.max())
            assert dx.max() <= 4 * EPS32 * (1.0 + wl.dt * umax), key
        for key in ("ux", "uy", "uz"):
            du = np.abs(gp[key][:n] - op[key])
            errs[key] = float(du.max())
            assert du.max() <= 8 * EPS32 * (umax + h * emax), key
        for d in range(3):
            err = np.abs(gF[6 + d] - o.F[6 + d])
            errs[f"J{'xyz'[d]}/max|J|"] = float(err.max() / np.max(np.abs(o.F[6 + d])))
            assert np.all(err <= (om.Jcnt[d] + 68) * EPS32 * om.Jabs[d] + 1e-300)
        for c, name in enumerate(("Ex", "Ey", "Ez", "Bx", "By", "Bz")):
            errs[name + "/max"] = float(np.max(np.abs(gF[c] - o.F[c])) / np.max(np.abs(o.F[c])))
        log(f"  mixed vs FP64 oracle, one step from S_{k}: {errs}")

    _run(wl, [0, 20], check)


def test_mixed_long_run_against_fp64_gpu():
    # 200 steps of the 64^3 x 50 ppc recipe at 16^3 x 20 ppc in both
    # precisions from the same (mixed-rounded) state: energies, total
    # momentum and the Gauss drift; the trajectories decorrelate (the plasma
    # is chaotic), so only ensemble quantities are compared
    wl = W.scaled(2, (16, 16, 16), 20, seed=45)
    sp = wl.species[0]
    o = _mixed_oracle(wl)
    xr = o.to_mixed([sp.x, sp.y, sp.z, sp.ux, sp.uy, sp.uz])
    sp.x, sp.y, sp.z, sp.ux, sp.uy, sp.uz = [np.ascontiguousarray(a) for a in xr]
    out = {}
    for prec in ("fp64", "mixed"):
        sim = pic.Simulation.from_workload(wl, precision=prec)
        try:
            d0 = sim.diagnostics()
            sim.step(200)
            d = sim.diagnostics()
            P = sim.particles(0)
            n = P["n"]
            mom = [float(np.sum(P[k][:n])) for k in ("ux", "uy", "uz")]
            absmom = [float(np.sum(np.abs(P[k][:n]))) for k in ("ux", "uy", "uz")]
            # the mean charge density is n0 = 1, so the Gauss drift is
            # relative to the density scale
            out[prec] = dict(WE=d[0], WB=d[1], K=d[2], Q=d[3], gauss=d[4], divB=d[5], mom=mom,
                             absmom=absmom, K0=d0[2])
        finally:
            sim.close()
    a, b = out["fp64"], out["mixed"]
    log(f"  200 steps, FP64: {a}")
    log(f"  200 steps, mixed: {b}")
    rel = {k: abs(a[k] - b[k]) / abs(a[k]) for k in ("WE", "WB", "K")}
    mom = [abs(a["mom"][d] - b["mom"][d]) / a["absmom"][d] for d in range(3)]
    log(f"  mixed vs FP64 after 200 steps: relative {rel}, momentum / sum|u| {mom}")
    assert a["Q"] == b["Q"]
    assert a["gauss"] <= 1e-12
    # FP32 rounding of J breaks exact continuity: a random walk, observed
    # 5.6e-8 of the density scale after 200 steps; bound 5e-6
    assert b["gauss"] <= 5e-6
    # observed about 1e-6 (W_E, W_B), 2e-8 (K) and 1e-8 of sum |u_d| (the
    # summed momentum); bounds about 100 times larger
    assert rel["WE"] <= 1e-4 and rel["WB"] <= 1e-4, rel
    assert rel["K"] <= 1e-6, rel
    assert max(mom) <= 1e-6, mom


def test_precision_variant_full_size_128c_32ppc():
    """The 128^3 x 32 ppc recipe (67,108,864 particles) in both precisions for
    200 steps from the same state (the mixed path's rounded state loaded into
    the FP64 context): charge, Gauss drift and the ensemble energies as in the
    16^3 run above, at the full size."""
    import torch
    wl = W.config4()
    n = wl.nparticles
    log(f"  precision variant at full size: {n} particles")
    dev = torch.device("cuda:0")
    keys = ("x", "y", "z", "ux", "uy", "uz", "id")
    out = {}
    state = None
    for prec in ("mixed", "fp64"):
        sim = pic.Simulation.from_workload(wl, precision=prec)
        try:
            if state is None:
                state = {k: torch.empty(n, dtype=torch.int64 if k == "id" else torch.float64,
                                        device=dev) for k in keys}
                pic.pic_get_particles(sim.ctx, 0, capacity=n, out=state)
                # the load's re-sort (a histogram scan over more than 2^24
                # entries) grouped the 67 M particles by supercell
                c = [torch.floor(state[k]).to(torch.int64) // wl.S for k in ("x", "y", "z")]
                ns = [v // wl.S for v in wl.n]
                sc = c[0] + ns[0] * (c[1] + ns[1] * c[2])
                assert bool(torch.all(sc[1:] >= sc[:-1]))
                assert int(torch.unique(state["id"]).numel()) == n
            else:
                sim.load_particles(0, *[state[k] for k in keys[:6]], state["id"])
            sim.step(200)
            d = sim.diagnostics()
            end = {k: torch.empty(n, dtype=torch.int64 if k == "id" else torch.float64,
                                  device=dev) for k in keys}
            pic.pic_get_particles(sim.ctx, 0, capacity=n, out=end)
            mom = [float(torch.sum(end[k])) for k in ("ux", "uy", "uz")]
            absmom = [float(torch.sum(torch.abs(end[k]))) for k in ("ux", "uy", "uz")]
            del end
            out[prec] = dict(WE=d[0], WB=d[1], K=d[2], Q=d[3], gauss=d[4], mom=mom,
                             absmom=absmom)
        finally:
            sim.close()
    a, b = out["fp64"], out["mixed"]
    log(f"  200 steps, FP64: {a}")
    log(f"  200 steps, mixed: {b}")
    rel = {k: abs(a[k] - b[k]) / abs(a[k]) for k in ("WE", "WB", "K")}
    mom = [abs(a["mom"][d] - b["mom"][d]) / a["absmom"][d] for d in range(3)]
    log(f"  mixed vs FP64 after 200 steps: relative {rel}, momentum / sum|u| {mom}")
    assert a["Q"] == b["Q"]
    assert a["gauss"] <= 1e-11
    # observed 4.4e-9 of the density scale; bound 5e-7
    assert b["gauss"] <= 5e-7
    # observed 1.2e-8 (W_E), 8.9e-8 (W_B), 1.1e-10 (K), about 2e-9 of
    # sum |u_d| (momentum); bounds about 100 times larger
    assert rel["WE"] <= 1e-6 and rel["WB"] <= 1e-5, rel
    assert rel["K"] <= 1e-8, rel
    assert max(mom) <= 2e-7, mom


@pytest.mark.parametrize("n,ppc", [((16, 16, 16), 64), ((8, 8, 8), 300)])
def test_mixed_dense_supercells_resort(n, ppc):
    # 4,096 and 19,200 particles per supercell: the neighbourhood re-sort
    # moves the packed arrays with the LDS-staged permutation (the second
    # case beyond its buffers); steps 19 (ends with the re-sort), 20, 21
    wl = W.scaled(2, n, ppc, seed=170 + ppc)
    _run(wl, [19, 20, 21], _against_mixed_oracle)


def test_mixed_dense_resort_with_particles_beyond_the_neighbouring_supercells():
    # the dense beam workload of test_gpu_parity (which checks that particles
    # end two supercells on): the neighbourhood re-sort gives way to the global
    # sort, whose order the push after it applies with the staged permutation
    _run(dense_beam_workload(), [19, 20, 21], _against_mixed_oracle)


def test_mixed_resort_with_particles_beyond_the_neighbouring_supercells():
    # a beam of every sixteenth particle at about 0.99 c crosses two 2-cell
    # supercells before the first re-sort: the global sort takes over (the
    # FP64 case in test_gpu_parity checks that the crossing happens)
    wl = W.plasma("beam-resort-mixed", (32, 16, 16), 2, 0.02, seed=52, noise=1e-2, S=2, R=10)
    sp = wl.species[0]
    rng = np.random.default_rng(53)
    sp.ux[3::16] = 6.0 + rng.random(len(sp.ux[3::16]))
    _run(wl, [9, 10, 19, 20], _against_mixed_oracle)
