"""Write the stored observed images of the parity and benchmark workloads.

Calls only the oracle (clean FP64 image of a seed-fixed truth) and the seeded input
generators (truth draw, PSF, noise). Run from the repository root:
    python tests/golden/make_workloads.py
Output: tests/golden/obs_<spec>_s<seed>.npy (float32, H x W) and truth_<spec>_s<seed>.npy.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def oracle_model(spec: synth.Spec) -> oracle.Model:  # noqa: D401
    return oracle.Model(H=spec.H, W=spec.W, k=spec.k, pix=spec.pix, epl=spec.epl,
                        shear=spec.shear, lens_light=spec.lens_light, nmax=spec.nmax,
                        psf=spec.psf.astype(np.float64), sigma_bkg=spec.sigma_bkg,
                        t_exp=spec.t_exp, gain=spec.gain)


def make(spec: synth.Spec, seed: int):
    truth = synth.draw_truth(spec, seed)
    clean = oracle.simulate(oracle_model(spec), truth.astype(np.float64))[0]
    obs = synth.add_noise(clean, seed, spec.sigma_bkg, spec.t_exp, spec.gain)
    np.save(os.path.join(OUT, f"obs_{spec.name}_s{seed}.npy"), obs)
    np.save(os.path.join(OUT, f"truth_{spec.name}_s{seed}.npy"), truth)
    return obs


if __name__ == "__main__":
    make(synth.spec_c1(), 0)
    for s in range(5):
        make(synth.spec_c2(), s)
    make(synth.spec_paper80(), 6)  # arc signal-to-noise 106, the paper's typical ~100
    print("ok")
