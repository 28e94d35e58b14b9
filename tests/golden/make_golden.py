"""Writes tests/golden/*.json from the FP64 oracle only (no GPU code).

c1_oracle_sample.json: I[f] of the 512-k parabolic-band case (one band,
m* = 0.3, 8^3 grid, q grid = k grid, Debye 5 km/s + Einstein 30/50 meV,
lognormal |g|^2, sigma = 8 meV, perturbed Fermi-Dirac f at 300 K) at the 12 states
of largest |I| and 4 evenly spaced ones, plus sum and max-abs over all states.  It pins the oracle
against accidental change; its correctness is pinned by tests/test_oracle.py.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    s = synth.parabolic_system(8)
    f = synth.c1_occupations(s)
    I = oracle.collision(s, f, s.nph(300.0))
    top = np.argsort(-np.abs(I), kind="stable")[:12]
    idx = np.unique(np.concatenate([top, np.linspace(0, s.n_states - 1, 4).astype(int)]))
    out = dict(description="oracle I[f] on the 512-k parabolic case; see make_golden.py",
               n_states=s.n_states, n_channels=s.n_channels,
               states=idx.tolist(), I=[float(I[i]) for i in idx],
               sum=float(I.sum()), max_abs=float(np.abs(I).max()))
    with open(os.path.join(HERE, "c1_oracle_sample.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
