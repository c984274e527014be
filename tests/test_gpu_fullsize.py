"""One-step oracle parity at the full sizes of the uniform workloads, in both
precisions, on the steps around a re-sort (Section 3: double precision, CIC,
VB; Section 4.3: supercells).

* 64^3 cells x 50 electrons (13,107,200 particles), FP64: step 19, which ends
  with the re-sort, and step 20, the push after it (the order is applied by
  the LDS-staged permutation at this density); FP32-mixed: steps 0 and 19.
* 128^3 cells x 32 electrons (67,108,864 particles): step 19 in FP64 and in
  mixed precision.  The re-sort there sorts 21-bit keys in two passes of 11-bit
  digits, whose histograms hold more than 2^24 entries (scanned in chunks with
  a carry); ids after it are compared with the oracle's order bit for bit.

The protocol and tolerances are those of gpu_parity_util (FP64) and
test_gpu_mixed (mixed: positions, momenta and ids bit for bit against the
oracle's mixed-precision loop, J, E and B within the reordering bound).
"""
import pytest

from paper_1608_01009_amd import workloads as W

from gpu_parity_util import log, one_step_parity
from test_gpu_mixed import _against_mixed_oracle, _run

pytestmark = pytest.mark.gpu


def test_64cubed_50ppc_fp64_resort_steps():
    wl = W.config2()
    log(f"  64^3 x 50 FP64: {wl.nparticles} particles, steps 19 and 20")
    reps, sim = one_step_parity(wl, [19, 20])
    assert int(sim.counters()[1]) >= 1          # a re-sort happened in between
    sim.close()


def test_64cubed_50ppc_mixed_steps_0_19():
    wl = W.config2()
    log(f"  64^3 x 50 mixed: {wl.nparticles} particles, steps 0 and 19")
    _run(wl, [0, 19], _against_mixed_oracle)


def test_128cubed_32ppc_fp64_resort_step():
    wl = W.config4()
    log(f"  128^3 x 32 FP64: {wl.nparticles} particles, step 19")
    reps, sim = one_step_parity(wl, [19])
    sim.close()


def test_128cubed_32ppc_mixed_resort_step():
    wl = W.config4()
    log(f"  128^3 x 32 mixed: {wl.nparticles} particles, step 19")
    _run(wl, [19], _against_mixed_oracle)
