"""Writes the FP64 oracle's Algorithm-2 solves that the full-schedule GPU parity tests compare
against (the oracle takes minutes on these sizes, longer than a test should wait).

Calls only the oracle and the seeded input generators.  Each file stores the final image, the
previous iterate (for the relative variation of the last iteration), the stopping quantities of
the final state, and the constants the GPU run must share (||phi||^2, gamma, step sizes), plus
a hash of the oracle sources and one of the generated inputs: tests/test_golden_files.py fails
when either changes after the file was written.

    python tests/golden/make_oracle_solves.py ring128 ring256
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import metrics, pd, problem  # noqa: E402
from paper_1801_02417_amd import workloads as wk  # noqa: E402

# name -> (workload, iterations per stage, power-iteration tolerance and bound)
SOLVES = {
    # the 128x128 ring + jet workload on its stated schedule: 2000 iterations = the
    # initialisation stage and 5 reweighting cycles (333 x 5 + 335)
    "ring128": (wk.ring128, pd.split_iterations(2000, 6), 1e-12, 1000),
    # the 256x256 workload the benchmark times: 300 iterations = 100 x (initialisation + 2 cycles)
    "ring256": (wk.ring256, [100, 100, 100], 1e-9, 300),
}


def oracle_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "oracle")
    for f in sorted(os.listdir(d)):
        if f.endswith(".py"):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def input_hash(wl) -> str:
    """Fingerprint of a generated workload: its sizes, truth, uv points and noise draws."""
    h = hashlib.sha256()
    h.update(repr((wl.n, wl.M, wl.taps, wl.oversample, wl.levels, wl.isnr_db)).encode())
    for a in (wl.truth, wl.uv, wl.noise):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


def golden_path(name: str) -> str:
    return os.path.join(HERE, f"oracle_{name}.npz")


def make(name: str) -> None:
    wl_fn, stages, rtol, max_iter = SOLVES[name]
    t0 = time.time()
    wl = wl_fn()
    b = problem.build(wl, norm_rtol=rtol, norm_max_iter=max_iter)
    print(f"{name}: built in {time.time() - t0:.1f} s, ||phi||^2 {b.phi_norm_sq:.12g}", flush=True)
    # Algorithm 2 with the last stage one iteration short, then that iteration: the final state
    # and the one before it (the oracle's iteration is a pure function of the state)
    short = list(stages)
    short[-1] -= 1
    st, gW, deltas = pd.alg2(b.pb, b.gamma, short, len(stages) - 1,
                             callback=lambda l, s: print(f"  stage {l} done at {time.time() - t0:.0f} s", flush=True))
    prev = st.S.copy()
    st = pd.alg1_iteration(st, b.pb, gW, "polsara")
    res = metrics.residual_norm(b.mop, st.S, b.pb.Y)
    _, zeta, n_p = metrics.polarization_error(b.mop, st.S, b.pb.Y)
    rv = metrics.relative_variation(st.S, prev)
    obj = metrics.weighted_l1(b.sara.adjoint, st.S, gW / b.gamma)
    snr = [metrics.snr_db(st.S[:, i], b.truth[:, i]) for i in range(4)]
    np.savez_compressed(golden_path(name), S=st.S, S_prev=prev, stages=np.array(stages), phi_norm_sq=b.phi_norm_sq,
                        gamma=b.gamma, steps=np.array([b.pb.tau, b.pb.rho1, b.pb.rho2, b.pb.rho3]), eps=b.pb.eps,
                        residual=res, zeta=zeta, n_p=n_p, rel_var=rv, objective=obj, deltas=np.array(deltas),
                        snr_db=np.array(snr), oracle_hash=oracle_hash(), input_hash=input_hash(wl))
    print(f"{name}: done in {time.time() - t0:.0f} s; SNR {['%.2f' % v for v in snr]} residual/eps {res / b.pb.eps:.6f} "
          f"N_p {n_p:.3f}", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or list(SOLVES):
        make(name)
