"""Write fluid_table_ne_1torr.json: the two-term transport table of the
synthetic neon cross sections (the striated 20 cm column's gas) on the
fluid model's uniform temperature grid.

E/N from 0.1 to 300 Td (200 values, log-spaced), solved by the project's
two-term Boltzmann solver, sorted by T_e = 2/3 mean energy and resampled
linearly onto T = FLUID_T_MIN + k FLUID_T_STEP (values below the lowest
solved temperature, 0.87 eV, take that row).  Columns as the fluid library
expects them: mu_e N, D_e N, mu_eps N, D_eps N, k_iz, L/N (section IV).

    python workloads/make_fluid_table.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import workloads as W                                   # noqa: E402
from paper_2202_03215_amd import closure as CL          # noqa: E402

NGAS_1TORR = 1.0 * 133.322368 / (1.380649e-23 * 300.0)


def main() -> int:
    EN = np.geomspace(1e-22, 3e-19, 200)
    T, cols = CL.transport_table(W.column_20cm(), EN, NGAS_1TORR)
    tab = CL.resample_uniform(T, cols, W.FLUID_T_MIN, W.FLUID_T_STEP, W.FLUID_T_LEN)
    out = dict(gas="Ne (synthetic cross sections)", EN_Td=[0.1, 300.0], n_EN=int(EN.size),
               T_solved_eV=[float(T.min()), float(T.max())], T_min=W.FLUID_T_MIN, T_step=W.FLUID_T_STEP,
               columns=["mu_e N", "D_e N", "mu_eps N", "D_eps N", "k_iz", "L/N"],
               table=[[float(v) for v in row] for row in tab])
    with open(os.path.join(HERE, "fluid_table_ne_1torr.json"), "w") as f:
        json.dump(out, f, indent=0)
    return 0


if __name__ == "__main__":
    sys.exit(main())
