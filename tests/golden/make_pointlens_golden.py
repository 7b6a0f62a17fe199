"""Write tests/golden/pointlens_born_ewald.json (calls only the oracle).

Born deflections through the periodic, neutralised point-mass potential (the
potential the FFT Poisson solver represents) for a sample of the static point-lens
rays above the resolution threshold theta_thresh = 4 cell / chi_l (paper Sec. 6.1,
Fig. 1 caption and text; Appendix D, Eq. pointmass_periodic for the periodic images).
Run from the repository root:  python tests/golden/make_pointlens_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import integrator, pointmass  # noqa: E402


def main():
    cfg = synth.pointlens()
    th0 = integrator.pixel_angles(cfg["ray_n"], cfg["ray_n"], cfg["fov"], cfg["fov"])
    chi_l = cfg["lens"][2] - cfg["observer"][2]
    thresh = 4.0 * cfg["box"] / cfg["mesh_n"] / chi_l
    r = np.linalg.norm(th0, axis=1)
    idx = np.where(r > thresh)[0][::17]
    be = pointmass.born_ewald(th0[idx], cfg["lens"], cfg["observer"], cfg["chi_s"], cfg["mass"], cfg["box"])
    thin = pointmass.thin_lens(th0[idx], chi_l, cfg["chi_s"], cfg["mass"])
    out = dict(
        source="oracle.pointmass.born_ewald; paper Sec. 6.1 and Appendix D (Eq. pointmass_periodic)",
        workload="static point lens: M=1e15 Msun/h, box 512 Mpc/h, 128^3 mesh, 64x64 rays over 10 deg",
        theta_thresh=thresh, ray_index=idx.tolist(), born_ewald=be.tolist(), thin_lens=thin.tolist())
    path = os.path.join(ROOT, "tests", "golden", "pointlens_born_ewald.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, len(idx), "rays")


if __name__ == "__main__":
    main()
