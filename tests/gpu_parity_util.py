"""Helpers of the GPU parity tests: one step from an identical state.

The GPU library advances k steps; its state S_k (particles in stored order
with ids, E, B) is read back; the oracle takes one step from S_k and its
result is compared with the GPU's S_{k+1}:
* ids (hence the stored order) and cell indices floor(x): bit for bit;
* x: within 2 ulp of the domain length (the push is evaluated in the same
  expression order on both sides, so in practice bit for bit);
* u, J, E, B: max |a - b| <= 1e-12 * max |b| per array.
"""
import math
import sys

import numpy as np

from gpu_layout import LayoutOracle
from paper_1608_01009_amd import pic

KEYS = ("x", "y", "z", "ux", "uy", "uz", "id")
REL_TOL = 1e-12


def dense_beam_workload():
    """6,400 particles per 4^3 supercell on 4 x 2 x 2 supercells (dense: a
    re-sort moves the data), every 32nd particle at about 0.99 c along x: it
    moves about 5.7 cells in the 20 steps before the first re-sort, and those
    starting in the last part of their supercell end two supercells on."""
    from paper_1608_01009_amd import workloads as W
    wl = W.scaled(2, (16, 8, 8), 100, seed=90)
    sp = wl.species[0]
    rng = np.random.default_rng(91)
    sp.ux[5::32] = 6.0 + rng.random(len(sp.ux[5::32]))
    return wl


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_for(wl):
    return LayoutOracle(wl.n, wl.dx, wl.dt, [(s.charge, s.mass, s.weight) for s in wl.species],
                        S=wl.S, R=wl.R)


def read_state(sim, nspecies):
    F = sim.fields()
    P = [sim.particles(s) for s in range(nspecies)]
    return F, P


def max_rel(a, b):
    scale = np.max(np.abs(b)) if b.size else 0.0
    d = np.max(np.abs(a - b)) if a.size else 0.0
    if scale == 0.0:
        return d
    return d / scale


def compare(gF, gP, o, L, tag="", rel_tol=REL_TOL, field_abs_floor=1e-300):
    """Compare GPU S_{k+1} with the oracle state after its step."""
    report = {}
    for s, gp in enumerate(gP):
        op = o.particles(s)
        n = gp["n"]
        assert n == len(op["x"]), f"{tag} species {s}: count {n} vs {len(op['x'])}"
        assert np.array_equal(gp["id"][:n], op["id"]), f"{tag} species {s}: order differs"
        for d, k in enumerate(("x", "y", "z")):
            g = gp[k][:n]
            w = op[k]
            assert np.array_equal(np.floor(g), np.floor(w)), f"{tag} species {s}: cell {k} differs"
            ulp = np.spacing(np.float64(L[d]))
            dx = np.max(np.abs(g - w)) if n else 0.0
            assert dx <= 2 * ulp, f"{tag} species {s}: {k} off by {dx}"
            report[f"s{s}.{k}.exact"] = float(np.mean(g == w)) if n else 1.0
        for k in ("ux", "uy", "uz"):
            r = max_rel(gp[k][:n], op[k])
            assert r <= rel_tol, f"{tag} species {s}: {k} rel {r}"
            report[f"s{s}.{k}.exact"] = float(np.mean(gp[k][:n] == op[k])) if n else 1.0
    names = ("Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz")
    for c, name in enumerate(names):
        r = max_rel(gF[c], o.F[c])
        if np.max(np.abs(o.F[c])) < field_abs_floor:
            r = np.max(np.abs(gF[c] - o.F[c]))
        assert r <= rel_tol, f"{tag} {name}: rel {r}"
        report[name] = float(r)
    return report


def one_step_parity(wl, ks, sim_kwargs=None, extra_check=None):
    """Run the GPU through the steps in ks (ascending); at each k compare the
    GPU's step k -> k+1 with the oracle's step from the GPU state S_k."""
    sim = pic.Simulation.from_workload(wl, **(sim_kwargs or {}))
    o = oracle_for(wl)
    nsp = len(wl.species)
    cur = 0
    reports = []
    try:
        for k in ks:
            log(f"  parity {wl.name}: advancing GPU to step {k}")
            if k > cur:
                sim.step(k - cur)
            F, P = read_state(sim, nsp)
            sim.step(1)
            cur = k + 1
            gF, gP = read_state(sim, nsp)
            o.set_state([[p[key][:p["n"]] for key in KEYS] for p in P], F[:6], k % wl.R)
            o.step(1)
            rep = compare(gF, gP, o, wl.n, tag=f"{wl.name} k={k}")
            if extra_check:
                extra_check(sim, k, rep)
            reports.append((k, rep))
            log(f"  parity {wl.name} k={k}: ok {rep}")
        return reports, sim
    except Exception:
        sim.close()
        raise
