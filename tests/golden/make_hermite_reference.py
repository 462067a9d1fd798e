"""Write the CPU-oracle reference of a Hermite block-step run.

Plummer N = 65536 (seed 2), eps = 1/256, eta = 0.01, dt_max = 1/16,
max_level = 30, integrated with 4th-order Hermite block steps to t = 1/8
by the CPU oracle (oracle.hermite with oracle.forces_f64).  Stores the
initial and final energy, the step and force-evaluation counts, the
per-step active counts, and the final state of 256 sampled particles.

    python tests/golden/make_hermite_reference.py [N] [out.json]

Uses only oracle/ and synth/.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from oracle import hermite as H  # noqa: E402


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 65536
    out = sys.argv[2] if len(sys.argv) > 2 else os.path.join(os.path.dirname(__file__),
                                                             f"hermite_plummer_N{n}.json")
    seed, eps2, eta, dt_max, max_level, t_end = 2, 2.0 ** -16, 0.01, 1.0 / 16, 30, 0.125
    p = synth.plummer(n, seed)

    def forces(x, v, m, act):
        a, j, ph, _ = oracle.forces_f64(x, v, m, eps2, act)
        return a, j, ph

    t0 = time.time()
    e0 = H.energy(p.pos, p.vel, p.mass, oracle.forces_f64(p.pos, p.vel, p.mass, eps2)[2])
    st = H.initialise(p.pos, p.vel, p.mass, eps2, eta, dt_max, max_level, forces)
    H.run_until(st, t_end, forces)
    e1 = H.energy(st.x, st.v, st.m, oracle.forces_f64(st.x, st.v, st.m, eps2)[2])
    rows = np.sort(np.random.default_rng(7).choice(n, 256, replace=False))
    doc = dict(
        workload=dict(kind="plummer", n=n, seed=seed, eps2=eps2, eta=eta, dt_max=dt_max, max_level=max_level,
                      t_end=t_end),
        E0=e0["E"], E1=e1["E"], K1=e1["K"], W1=e1["W"], drift=abs(e1["E"] - e0["E"]) / abs(e0["E"]),
        steps=st.steps, force_evals=st.force_evals, clamps=st.clamps,
        n_active=st.n_active_hist,
        sample_rows=rows.tolist(), sample_pos=st.x[rows].tolist(), sample_vel=st.v[rows].tolist(),
        sample_level=st.level[rows].tolist(),
        level_histogram=np.bincount(st.level, minlength=max_level + 1).tolist(),
        cpu_seconds=round(time.time() - t0, 1),
        generator="tests/golden/make_hermite_reference.py (oracle.hermite + oracle.forces_f64)")
    with open(out, "w") as f:
        json.dump(doc, f)
    print(f"wrote {out}: steps={st.steps} evals={st.force_evals} drift={doc['drift']:.3e} "
          f"in {doc['cpu_seconds']} s", flush=True)


if __name__ == "__main__":
    main()
