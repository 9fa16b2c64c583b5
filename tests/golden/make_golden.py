"""Write tests/golden/oracle_small.json from the CPU oracle (and nothing else).

Run from the repository root:  python tests/golden/make_golden.py
The stored values guard the oracle against unintended changes of its
arithmetic; they are outputs of oracle/ on inputs from synthetic_inputs.
"""
import json
import pathlib
import sys

HERE = pathlib.Path(__file__).resolve().parent
sys.path.insert(0, str(HERE.parent.parent))
sys.path.insert(0, str(HERE.parent))

import oracle  # noqa: E402
import golden_io  # noqa: E402


def main():
    lib = oracle.load()
    cases = []
    for name, method, dims, seed, ghost, a, b, g, sweeps in golden_io.CASES:
        case = dict(name=name, method=method, dims=list(dims), seed=seed, ghost=ghost, a=a, b=b,
                    g=g, sweeps=sweeps)
        out = golden_io.run_case(case, lib)
        case["shape"] = list(out.shape)
        case["expected_hex"] = [float(v).hex() for v in out.ravel()]
        cases.append(case)
    doc = {"source": "oracle/oracle.c via tests/golden/make_golden.py; inputs from "
                     "synthetic_inputs.uniform_padded / uniform_rhs",
           "definition": "Sec. 3 Jacobi and Gauss-Seidel loop nests, FP64, operand order "
                         "((((x- + x+) + y-) + y+) + z-) + z+, then (a*c) + (b*s) [+ g*f]",
           "cases": cases}
    golden_io.GOLDEN.write_text(json.dumps(doc, indent=1) + "\n")
    print("wrote", golden_io.GOLDEN)


if __name__ == "__main__":
    main()
