"""Write the Maxwell coexistence table used by the seeded input generators.

TEST INFRASTRUCTURE (oracle script).  Calls only ``oracle.eos``.  The table
lists (T/T_c, rho_l, rho_g) for the Carnahan-Starling EOS with b = 4, R = 1
and T_c = 0.094 a (the rounded critical temperature the paper uses in
Sec. IV.A and IV.C).  With b fixed the Maxwell densities depend only on T/T_c,
not on a (p_EOS scales with a at fixed T/T_c).

Usage:  python -m oracle.make_coexistence_table   (from the repository root)
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import eos

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "workloads", "coexistence_table.json")
TC_PER_A = 0.094


def main():
    rows = []
    for tb in np.round(np.arange(0.40, 0.9501, 0.0025), 6):
        rl, rg = eos.maxwell(float(tb) * TC_PER_A * 1.0, 1.0, 4.0, 1.0)
        rows.append([float(tb), rl, rg])
    doc = {
        "what": "Maxwell equal-area coexistence densities of the Carnahan-Starling EOS",
        "b": 4.0, "R": 1.0, "Tc_per_a": TC_PER_A,
        "columns": ["T_over_Tc", "rho_l", "rho_g"],
        "rows": rows,
        "generator": "python -m oracle.make_coexistence_table",
    }
    body = json.dumps({k: v for k, v in doc.items() if k != "rows"}, indent=1)[:-2]
    rows_txt = ",\n  ".join(json.dumps(r) for r in rows)
    with open(OUT, "w") as fh:
        fh.write(body + ',\n "rows": [\n  ' + rows_txt + "\n ]\n}\n")
    print(f"wrote {len(rows)} rows to {OUT}")


if __name__ == "__main__":
    main()
