"""Write the placeholder table of the 209 IMRPhenomD-structured fit coefficients.

The model calibrates 19 phenomenological parameters, each a fit in the symmetric mass
ratio eta and the effective PN spin chi_PN with 11 terms (19 x 11 = 209 coefficients,
paper Sec. 3.1).  The published calibrated values are not available to this project, so
this script writes a *placeholder* table instead: for every parameter a central value
that gives a physically sensible waveform shape near equal mass and zero spin, plus
small seeded variations on the other ten basis terms so that every one of the 209
coefficients is non-zero and influences the waveform.

Basis order of the 11 terms (x = chi_PN - 1):
    1, eta, x, x*eta, x*eta^2, x^2, x^2*eta, x^2*eta^2, x^3, x^3*eta, x^3*eta^2
Parameter order of the 19 rows:
    rho1 rho2 rho3 v2 gamma1 gamma2 gamma3 sigma1 sigma2 sigma3 sigma4
    beta1 beta2 beta3 alpha1 alpha2 alpha3 alpha4 alpha5

Run:  python paper_2302_05329_amd/data/make_lambda_placeholder.py
It rewrites phenomd_lambda_placeholder.txt next to this file (deterministic, seed 2302).
"""
import os

import numpy as np

NAMES = ["rho1", "rho2", "rho3", "v2", "gamma1", "gamma2", "gamma3",
         "sigma1", "sigma2", "sigma3", "sigma4", "beta1", "beta2", "beta3",
         "alpha1", "alpha2", "alpha3", "alpha4", "alpha5"]

# Value of each parameter at the anchor point eta = 1/4, chi_PN = 0 (x = -1).
CENTRAL = [3900.0, -25000.0, 50000.0, 0.80, 0.0069, 0.80, 0.70,
           2000.0, -10000.0, 22000.0, -14000.0, 97.0, -2.8, -1.6e-5,
           43.0, -0.07, -0.16, 0.77, 0.99]

# Relative size of the ten non-constant basis terms (x is in [-1.9, -0.1] for |chi|<=0.9).
REL = np.array([0.40, 0.05, 0.10, 0.20, 0.02, 0.04, 0.08, 0.005, 0.01, 0.02])


def basis(eta, chi_pn):
    x = chi_pn - 1.0
    return np.array([1.0, eta, x, x * eta, x * eta**2, x**2, x**2 * eta, x**2 * eta**2,
                     x**3, x**3 * eta, x**3 * eta**2])


def make_table(seed=2302):
    rng = np.random.Generator(np.random.PCG64(seed))
    table = np.zeros((19, 11))
    b0 = basis(0.25, 0.0)
    for i, c in enumerate(CENTRAL):
        signs = rng.choice([-1.0, 1.0], size=10)
        rel = REL * signs * rng.uniform(0.5, 1.0, size=10)
        row = np.zeros(11)
        row[1:] = c * rel
        # constant term chosen so that the fit returns exactly `c` at the anchor point
        row[0] = c - float(np.dot(row[1:], b0[1:]))
        table[i] = row
    return table


def main():
    table = make_table()
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "phenomd_lambda_placeholder.txt")
    with open(path, "w") as fh:
        fh.write("# PLACEHOLDER IMRPhenomD-structured fit coefficients (not the published calibration).\n")
        fh.write("# Written by make_lambda_placeholder.py, seed 2302. 19 rows x 11 columns.\n")
        fh.write("# rows: " + " ".join(NAMES) + "\n")
        fh.write("# cols: 1 eta x x*eta x*eta^2 x^2 x^2*eta x^2*eta^2 x^3 x^3*eta x^3*eta^2  (x = chi_PN - 1)\n")
        for name, row in zip(NAMES, table):
            fh.write(" ".join(repr(float(v)) for v in row) + f"  # {name}\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
