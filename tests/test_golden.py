"""Stored fixtures: the seeded inputs and the oracle's values have not drifted.

The fixtures are written by ``tests/golden/make_golden.py`` from the input
generator and the oracle only."""

import json
import os

import numpy as np

import oracle as O
from paper_1812_06765_amd import synth

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    with open(os.path.join(HERE, name)) as f:
        return json.load(f)


def test_inputs_unchanged():
    want = _load("inputs.json")
    p = synth.blob_phantom_pair((32, 32, 32), seed_R=1, seed_u=2, max_disp=2.0)
    assert synth.sha256(p.R) == want["blob32_R"]
    assert synth.sha256(p.T) == want["blob32_T"]
    c = synth.ct_phantom_pair((64, 64, 64), seed_R=3, seed_u=4)
    assert synth.sha256(c.R) == want["ct64_R"]
    assert synth.sha256(c.T) == want["ct64_T"]
    d = synth.smooth_node_perturbation((17, 17, 17), 8.0, 1.5, seed=7)
    assert synth.sha256(d) == want["pert17"]
    assert [list(s) for s in synth.batch_shapes()] == want["batch_shapes"]


def test_oracle_values_unchanged():
    want = _load("oracle_values.json")
    p = synth.blob_phantom_pair((32, 32, 32), seed_R=1, seed_u=2, max_disp=2.0)
    prob = O.Problem(p.R, p.T, (1.0, 1.0, 1.0), (17, 17, 17), 0.1, 0.1, 0.1)
    d = synth.smooth_node_perturbation(prob.my, 8.0, 1.5, 7)
    for name, y in (("identity", prob.identity().astype(np.float32)),
                    ("perturbed", (prob.identity() + d).astype(np.float32))):
        assert synth.sha256(y) == want[name]["y_sha256"]
        J, g, (D, S) = O.eval_J_grad(prob, y)
        for k, v in (("J", J), ("D", D), ("S", S), ("grad_l2", float(np.linalg.norm(g)))):
            assert abs(v - want[name][k]) <= 1e-12 * max(1.0, abs(want[name][k])), (name, k)
