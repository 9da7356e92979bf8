"""Checks of the stored full-length FP64 oracle runs (CPU only).

* The adjoint workload (96^3, 27 cubes) runs with the fixed balance
  acceleration (balance mode 1), which the adjoint supports: over its 500
  steps the lattice momentum drifts by less than 1e-3 of the particles' mean
  settling velocity (per unit mass), so the settling is that of a box with
  zero net volume flow to that accuracy.
* The dense boxes run with the zero-net-flux controller (balance mode 2):
  after 1000 steps the mean fluid velocity is below 1e-3 of the mean
  settling velocity.
* The walled box (128^3, 121 cubes, 2000 steps) has cubes reaching the
  bottom wall: contacts with the wall start and carry a force.
"""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_fullrun_refs as R  # noqa: E402


def _ref(name):
    if not os.path.exists(R.ref_path(name)):
        pytest.skip(f"no stored oracle run for {name}")
    return np.load(R.ref_path(name))


def _drift(d):
    """|lattice momentum| / lattice mass over |mean particle U_z| at the end."""
    return np.abs(d["momentum"]).max() / d["mass"] / abs(d["snap_U"][-1][:, 2].mean())


def test_adjoint_box_balance_drift():
    d = _ref("C5")
    assert int(d["steps"]) == 500
    assert _drift(d) < 1e-3
    # no node is flagged by the rough detection in any step
    assert not d["det_n"].any() and len(d["episodes"]) == 0


@pytest.mark.parametrize("name", ["C3", "C4"])
def test_dense_boxes_hold_zero_net_flow(name):
    d = _ref(name)
    assert int(d["steps"]) == 1000
    assert _drift(d) < 1e-3


def test_walled_box_wall_contacts():
    d = _ref("C2")
    assert int(d["steps"]) == 2000
    ep = d["episodes"]
    assert (ep[:, 1] < 0).any()
    # stored references are consistent: snapshot steps and step records
    assert d["snap_steps"][0] == 0 and d["snap_steps"][-1] == 2000
    assert d["act_n"].shape == (2001,)
