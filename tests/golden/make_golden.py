"""Write the golden fixtures in this folder.

The paper prints no worked numeric example, so the fixtures here are:

* ``inputs.json``: SHA-256 digests of the seeded synthetic inputs, so that a
  change of the generator cannot go unnoticed;
* ``oracle_values.json``: J, D and S of the oracle on the 32^3 blob pair (the
  single-level workload of Sec. 3's smallest resolution) at the identity and
  at a fixed smooth perturbation, so that a change of the oracle's arithmetic
  cannot go unnoticed.

Only the input generator and ``oracle/`` are called.  Run from the repository
root:  python tests/golden/make_golden.py
"""

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1812_06765_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def inputs():
    out = {}
    p = synth.blob_phantom_pair((32, 32, 32), seed_R=1, seed_u=2, max_disp=2.0)
    out["blob32_R"] = synth.sha256(p.R)
    out["blob32_T"] = synth.sha256(p.T)
    c = synth.ct_phantom_pair((64, 64, 64), seed_R=3, seed_u=4)
    out["ct64_R"] = synth.sha256(c.R)
    out["ct64_T"] = synth.sha256(c.T)
    d = synth.smooth_node_perturbation((17, 17, 17), 8.0, 1.5, seed=7)
    out["pert17"] = synth.sha256(d)
    out["batch_shapes"] = synth.batch_shapes()
    return out


def perturbed_y(prob, seed=7, amp=1.5):
    d = synth.smooth_node_perturbation(prob.my, 8.0, amp, seed)
    return (prob.identity() + d).astype(np.float32)


def oracle_values():
    p = synth.blob_phantom_pair((32, 32, 32), seed_R=1, seed_u=2, max_disp=2.0)
    prob = O.Problem(p.R, p.T, (1.0, 1.0, 1.0), (17, 17, 17), 0.1, 0.1, 0.1)
    out = {}
    for name, y in (("identity", prob.identity().astype(np.float32)),
                    ("perturbed", perturbed_y(prob))):
        J, g, (D, S) = O.eval_J_grad(prob, y)
        out[name] = {"J": J, "D": D, "S": S, "grad_l2": float(np.linalg.norm(g)),
                     "y_sha256": synth.sha256(y)}
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "inputs.json"), "w") as f:
        json.dump(inputs(), f, indent=1, sort_keys=True)
    with open(os.path.join(HERE, "oracle_values.json"), "w") as f:
        json.dump(oracle_values(), f, indent=1, sort_keys=True)
    print("written")
