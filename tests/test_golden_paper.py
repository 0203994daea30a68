"""Values printed in the paper, stored with their citations in
tests/golden/paper_values.json, checked against the oracle and inputs."""
import json
import math
import os

import numpy as np

import synth
from oracle import rollout as ro
from oracle import smc
from tests.oracle_helpers import mini

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_objective_weights_table():
    t = GOLD["objective_weights"]
    dep, arr = t["departure"], t["arrival"]
    w = synth.MIX_WEIGHTS
    assert (w[0], w[1], w[2]) == (arr["flowfield_heading"], arr["nominal_altitude"], arr["fuel"])
    assert (w[3], w[4], w[5], w[6]) == (dep["bearing"], dep["fuel"], dep["altitude"], dep["airspeed"])
    assert abs(sum(dep.values()) - 1) < 1e-12 and abs(sum(arr.values()) - 1) < 1e-12


def test_schedule_from_printed_constants():
    g = GOLD["sample_schedule"]
    for J in range(g["J_max"] + 1):
        assert smc.sample_schedule(J) == math.floor(g["a"] + g["b"] * math.exp(g["rate"] * J))


def test_bearing_example():
    g = GOLD["bearing_example"]
    s = mini(N=1, kinds=[1])
    s["cost_w"] = np.array([0, 0, 0, 1.0, 0, 0, 0, 0, 0])
    thF = s["targets"][0, 0]
    for off, J in ((0.0, g["on_bearing_J"]), (math.pi / 2, g["ninety_off_J"])):
        c = ro.step_cost(s, 3, 9e3 * math.cos(thF + off), 9e3 * math.sin(thF + off),
                         2000.0, 200.0, 0.0, 400.0)
        assert abs((1.0 - float(np.ravel(c)[0])) - J) < 1e-15
