"""Writes workloads/neural_calibration.json: the scale constants of each seeded
neural bound, computed in FP64 by the oracle (oracle.sdb.calibrate_network).

Run from the repository root:  python tests/golden/calibrate_neural.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W                 # noqa: E402
from oracle.sdb import calibrate_network  # noqa: E402


def networks():
    """(seed, width, depth, n_freq, activation) of every network the workloads use."""
    nets = [(0, 256, 4, 16, "softplus"), (0, 64, 4, 16, "softplus"), (0, 128, 4, 16, "softplus"),
            (0, 64, 8, 0, "relu")]
    for s in W.batch_scenes():
        if s["kind"] == "mlp":
            nets.append((s["seed"], s["width"], 4, 16, "softplus"))
    return sorted(set(nets))


def main():
    probe = W.probe_points()
    out = {}
    for (seed, width, depth, nf, act) in networks():
        net = W.mlp_net(seed, width, depth, nf, act)
        c = calibrate_network(net, probe, W.NEURAL_AMPLITUDE, W.NEURAL_R0)
        out[W.calibration_key(seed, width, depth, nf, act)] = c
        print(seed, width, depth, nf, act, c, flush=True)
    with open(W.neural_calibration_path(), "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
