"""Writes sigma_star_cs.json: the theory sigma* of the improved scheme for the
C-S EOS (a=1, b=4, R=1, G=-1) on a T/Tc grid.  sigma* makes the solution of
the mechanical stability condition (Eq. 26, eps = 16 sigma, Sec. IV.B) have
the Maxwell vapour density (Eq. 7).  Calls only the oracle."""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import numpy as np  # noqa: E402

from oracle import thermo as th  # noqa: E402

if __name__ == "__main__":
    grid = [round(float(t), 4) for t in np.arange(0.60, 0.9501, 0.025)]
    out = {"_about": __doc__, "t_over_tc": grid,
           "sigma_star": [th.sigma_star_cs(t) for t in grid],
           "maxwell_rho_l": [th.maxwell_cs(t).rho_l for t in grid],
           "maxwell_rho_g": [th.maxwell_cs(t).rho_g for t in grid]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sigma_star_cs.json")
    json.dump(out, open(path, "w"), indent=1)
    print(path)
