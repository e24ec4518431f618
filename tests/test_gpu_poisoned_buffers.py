"""Results must not depend on what freshly allocated device memory held.

With GOTHIC_POISON_ALLOC set, the library fills every new floating-point
buffer with all-ones bytes (NaN) before first use, so a kernel that reads a
value no kernel of the evaluation wrote shows up here.  The cases cover the
whole pipeline of one evaluation: node moments with monopole and quadrupole
terms (the internal-node pass reads the root record, written last, from
lanes that have no child), groups and their balls, the walk with both
multipole MACs, batched systems, block steps and the float64 direct sum.
"""
from __future__ import annotations

import numpy as np
import pytest

import ics
import oracle
import test_gpu_balls as balls_tests
import test_gpu_batched as batched_tests
import test_gpu_direct as direct_tests
import test_gpu_mac as mac_tests
import test_gpu_parity as parity_tests
import test_gpu_sim as sim_tests
from gpu_util import run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def poisoned(monkeypatch):
    monkeypatch.setenv("GOTHIC_POISON_ALLOC", "1")


@pytest.mark.parametrize("multipole", [1, 2])
def test_node_records_are_all_written(multipole):
    # every node record is a function of the particles alone: finite, and
    # equal to the float64 moments of the oracle's tree
    x = ics.nfw(20000, seed=23)
    ctx, out = run_gpu(x, 1 / 128, 0.5, multipole=multipole, r_crit=0.0)
    assert np.all(np.isfinite(out))
    com, b, q = ctx.nodes()
    assert np.all(np.isfinite(com)) and np.all(np.isfinite(b)) and np.all(np.isfinite(q))
    ks, perm, _ = ctx.keys()
    t = oracle.build(ks, 16)
    com_o, b_o, _ = oracle.moments(t, x[perm].astype(np.float64))
    scale = np.abs(com_o[:, :3]).sum(1) + b_o
    assert np.all(np.abs(com[:, :3] - com_o[:, :3]).max(1) <= 2e-6 * scale + 1e-30)
    assert np.all(np.abs(b - b_o) <= 1e-5 * b_o + 2e-6 * scale)


@pytest.mark.parametrize("multipole", [1, 2])
def test_forces_without_a_gap_split(multipole):
    parity_tests._check_forces(ics.nfw(20000, seed=23), 1 / 128, 0.5, multipole=multipole,
                               r_crit=0.0)


def test_forces_of_an_active_subset():
    x = ics.nfw(30000, seed=16)
    parity_tests._check_forces(x, 1 / 128, 0.5, active=ics.random_active(30000, 0.2, seed=17))


def test_each_ball_kind():
    for name in ("SEB", "EBS", "COM", "CMP"):
        balls_tests.test_forces_with_each_ball(name)


def test_both_multipole_macs():
    mac_tests.test_acceleration_mac(2.0 ** -7, 2)
    mac_tests.test_multipole_mac(1e-2, 2)


def test_batched_systems():
    batched_tests.test_batched_equals_single_system_calls(2)


def test_block_steps():
    sim_tests.test_block_steps_match_oracle(False)


def test_direct_sum():
    direct_tests.test_direct_sampled_targets_ragged_chunks()
