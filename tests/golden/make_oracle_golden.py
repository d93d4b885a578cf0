"""Write oracle_small_fields.txt: the oracle's P_min / P_max on small seeded
FP64 fields of each closed-form model (a regression fixture: it calls only
the oracle and the seeded generators).  Run from the repository root:
    python tests/golden/make_oracle_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402

CASES = [("uniform", 0, 4, 5, 0), ("epanechnikov", 1, 4, 5, 0), ("histogram", 2, 4, 5, 4)]


def main():
    lines = ["# oracle P_min / P_max (FP64, float.hex) on seeded fields; written by make_oracle_golden.py",
             "# case model_id H W nbins seed width"]
    for name, model, H, W, nb in CASES:
        seed, width = 40 + model, 0.3
        p = workloads.random_params(model, seed, H, W, nbins=max(nb, 1), width=width)
        pmin, pmax = oracle.forward(model, p)
        lines.append(f"case {name} {model} {H} {W} {nb} {seed} {width}")
        lines.append("p_min " + " ".join(float(v).hex() for v in pmin.ravel()))
        lines.append("p_max " + " ".join(float(v).hex() for v in pmax.ravel()))
    with open(os.path.join(HERE, "oracle_small_fields.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
