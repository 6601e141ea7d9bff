"""Writes the stored oracle runs used by the full-size GPU tests.

Each file holds the design and outputs of one adaptive run of the oracle
(plain FP64 C, `oracle/`) at a workload's full size: the cycle ends t_l, the
M-phase lengths R_l, the accepted-move counts of every Metropolis step, and
the log marginal likelihood with its NSE (Section 4.2).  Only `oracle/` and
the input generator `synthdata/` are called.  Run from the repository root:
`python tests/golden/write_oracle_runs.py [workload ...]` (default: all).
The EGARCH(2) Student-t run takes about an hour on eight host threads.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synthdata as SD  # noqa: E402

RUNS = [("egarch11", 1), ("egarch2t", 1)]


def main(names):
    for name, seed in RUNS:
        if names and name not in names:
            continue
        w = SD.workload(name)
        om = O.Model.from_workload(w)
        rc, rec, _ = O.run(om, w.J, w.N, seed, check_every=1, Lmax=2048, RmaxRec=64)
        assert rc == 0, rc
        s = rec.summary()
        L = int(s["L"])
        out = {
            "workload": name, "J": w.J, "N": w.N, "T": w.T, "seed": seed,
            "t_end": [int(x) for x in s["t_end"][:L]],
            "R": [int(x) for x in s["R"][:L]],
            "n_accept": [[int(x) for x in rec.n_acc[l][:int(s["R"][l])]] for l in range(L)],
            "log_ml": float(s["log_ml"]), "nse": float(s["nse"]),
            "log_ml_tilde": float(s["log_ml_tilde"]),
        }
        path = os.path.join(HERE, f"oracle_run_{name}_seed{seed}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(path, L, out["log_ml"], out["nse"], flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
