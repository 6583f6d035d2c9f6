"""Writes tests/golden/sysid64_oracle.npz: FP64 oracle results for the
64-instance system-identification batch (64^3 grids, N_i ~ U[20k, 200k], seed
4), which the GPU parity tests compare the batched FP32 path against.

  * states after 200 sub-steps of four instances (the smallest, the largest
    and two seeded others), on a seeded sample of 1024 particles each (the
    oracle has to run every particle; only the sample is stored);
  * the loss and the 9-parameter forward-mode gradient of the smallest
    instance after the full 500 sub-steps.

It calls only the oracle and the input generators, one process per case
(about 10 minutes on 8 cores).  Run from the repository root:
    python tests/golden/make_sysid64_oracle.py
"""
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sysid64_oracle.npz")
STATE_STEPS = 200
GRAD_STEPS = 500
SAMPLE = 1024


def sampled_instances(ws, n_random=2, seed=9):
    """Smallest, largest and n_random seeded other instances of a batch."""
    ns = [w.n_particles for w in ws]
    picks = [int(np.argmin(ns)), int(np.argmax(ns))]
    rest = [i for i in range(len(ws)) if i not in picks]
    rng = np.random.default_rng(seed)
    picks += [int(i) for i in rng.choice(rest, n_random, replace=False)]
    return picks


def particle_sample(n, i):
    return np.sort(np.random.default_rng(1000 + i).choice(n, SAMPLE, replace=False))


def state_case(i):
    w = W.sysid_batch(64, steps=STATE_STEPS)[i]
    r = oracle.rollout(oracle.config(w), w.params, oracle.initial_state(W.bed_positions(w)), STATE_STEPS)
    assert r["stats"][0] == 0 and r["stats"][4] == 0, r["stats"]
    idx = particle_sample(w.n_particles, i)
    return i, idx, r["state"][idx]


def grad_case(i):
    w = W.sysid_batch(64, steps=GRAD_STEPS)[i]
    r = oracle.rollout(oracle.config(w), w.params, oracle.initial_state(W.bed_positions(w)), GRAD_STEPS,
                       target=W.target_heightmap(w), grad=True)
    assert r["stats"][0] == 0 and r["stats"][4] == 0, r["stats"]
    return i, r["loss"], r["grad"]


def main():
    oracle.build(force=True)
    ws = W.sysid_batch(64, steps=GRAD_STEPS)
    picks = sampled_instances(ws)
    smallest = picks[0]
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        g = ex.submit(grad_case, smallest)
        states = list(ex.map(state_case, picks))
        gi, loss, grad = g.result()
    out = {"state_steps": np.array(STATE_STEPS), "grad_steps": np.array(GRAD_STEPS),
           "instances": np.array([s[0] for s in states]),
           "grad_instance": np.array(gi), "loss": np.array(loss), "grad": grad}
    for i, idx, st in states:
        out[f"idx_{i}"] = idx.astype(np.int64)
        out[f"state_{i}"] = st
    np.savez_compressed(OUT, **out)
    print(f"wrote {OUT}: instances {picks}, grad of {gi}: loss {loss}, grad {grad}")


if __name__ == "__main__":
    main()
