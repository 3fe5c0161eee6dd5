"""Plain FP64 CPU oracle for the IMRPhenomD-structured waveform and the products built on it.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module: only the
tests, the package smoke check and the benchmark's CPU-baseline leg do.  It shares no
code with the GPU library; the two meet only in the seeded inputs.

What it computes (paper: Sec. 2 and Sec. 3; the model itself is the aligned-spin
IMRPhenomD of Husa et al. 2016 / Khan et al. 2016, which the paper uses but does not
print, so its structure is restated here from those model papers):

  * source map        theta -> (M, eta, delta, chi1, chi2, D, tc, phic)
  * coefficient fits  Lambda_i = sum_k lambda[i][k] B_k(eta, chi_PN)      (Sec. 3.1: 209 numbers)
  * final state       final spin, radiated energy, ring-down and damping frequencies
  * phase             inspiral (TaylorF2 3.5PN + pseudo-PN sigma terms), intermediate,
                      merger-ringdown; joined C1 at Mf = 0.018 and Mf = f_RD / 2 (Sec. 3.1)
  * amplitude         inspiral (PN + rho terms), intermediate quartic (5 conditions),
                      merger-ringdown Lorentzian; joined C1 at Mf = 0.014 and f_peak
  * strain            h(f) = A(f) exp(-i Psi(f)), zero above Mf = 0.2
  * inner product     Eq. 1 as a Riemann sum on the grid; likelihood ln L = (d|h) - (h|h)/2
  * Fisher matrix     Eq. 8: F_ij = (d_i h | d_j h)
  * match / mismatch  max over lag (discrete FFT lag) and phase (modulus), Eqs. 2-4
  * coefficient fit   one gradient-descent step on the mean mismatch over targets, Eqs. 6-7
  * derivatives       complex-step differentiation of the real amplitude and phase
                      (a technique unrelated to the GPU's hand-written tangents)

Where the paper is silent, the reading taken is stated at the point of use.

Parity pins (tests/test_oracle_pins.py): C1 continuity at every join, the leading
TaylorF2 term and its O(v^2) residual, the non-spinning TaylorF2 coefficients derived
independently from PN energy and flux, the Newtonian amplitude limit, exact 1/D
scaling, exact linear tc/phic terms, m1<->m2 swap symmetry, Fisher closed forms and
positive definiteness, gradients against central differences, noise-free likelihood
stationarity, FFT match against a brute-force DFT, lag invariance and total-mass
invariance of the match on an Mf grid with a flat PSD, the first-order decrease of the mean
mismatch under a small descent step.
The spin-orbit parts of the phase coefficients (1.5, 2.5, 3 and 3.5PN) and the 2PN spin-spin
terms (the two bodies' interaction, and each body's spin squared through the Kerr test-mass
limit) are pinned by derivations from the spinning binding energy and flux.
Parity unpinned (model fidelity): the 3PN spin-spin phase terms, the spin parts of the PN
amplitude coefficients and those beyond 1PN, the final-spin / radiated-energy / ring-down
stand-ins and the placeholder coefficient table — nothing available here fixes their
published values.
"""
import math

import numpy as np

# ---- constants (the paper is silent; IAU 2015 nominal values) ----------------------
C_SI = 299792458.0
GM_SUN = 1.3271244e20
T_SUN = GM_SUN / C_SI**3          # 4.925490947641267e-06 s
MPC_M = 3.0856775814913673e22
EULER_GAMMA = 0.57721566490153286061

F_AMP_JOIN = 0.014    # amplitude: inspiral -> intermediate (Mf)
F_PHASE_JOIN = 0.018  # phase: inspiral -> intermediate (Mf)
F_CUT = 0.2           # the model is zero above Mf = 0.2

PARAM_MC_ETA = 0
PARAM_LNMC_ETA_LND = 1
PARAM_MC_Q = 2
PARAM_M1M2 = 3

LAMBDA_NAMES = ["rho1", "rho2", "rho3", "v2", "gamma1", "gamma2", "gamma3",
                "sigma1", "sigma2", "sigma3", "sigma4", "beta1", "beta2", "beta3",
                "alpha1", "alpha2", "alpha3", "alpha4", "alpha5"]


# ====================================================================================
# source parameters
# ====================================================================================

def source(theta, param):
    """theta (7 numbers) -> dict of intrinsic/extrinsic source quantities.

    Works for complex-step perturbed theta.  delta = (m1 - m2)/M keeps its sign, so an
    unsorted (m1, m2) pair maps to the swapped binary consistently.
    """
    t = list(theta)
    if param == PARAM_MC_ETA:
        mc, eta = t[0], t[1]
        mt = mc * eta ** (-0.6)
        delta = (1.0 - 4.0 * eta) ** 0.5
        dist = t[4]
    elif param == PARAM_LNMC_ETA_LND:
        mc, eta = np.exp(t[0]), t[1]
        mt = mc * eta ** (-0.6)
        delta = (1.0 - 4.0 * eta) ** 0.5
        dist = np.exp(t[4])
    elif param == PARAM_MC_Q:
        mc, q = t[0], t[1]
        eta = q / (1.0 + q) ** 2
        mt = mc * eta ** (-0.6)
        delta = (1.0 - q) / (1.0 + q)
        dist = t[4]
    elif param == PARAM_M1M2:
        m1, m2 = t[0], t[1]
        mt = m1 + m2
        eta = m1 * m2 / mt**2
        delta = (m1 - m2) / mt
        mc = mt * eta**0.6
        dist = t[4]
    else:
        raise ValueError(f"unknown parameterisation {param}")
    return dict(M=mt, eta=eta, delta=delta, Mc=mc, chi1=t[2], chi2=t[3], D=dist,
                tc=t[5], phic=t[6])


def domain_ok(theta, param):
    """Physical domain of the model: finite, masses > 0, 0 < eta <= 1/4, |chi| <= 1, D > 0."""
    t = np.asarray(theta, dtype=np.float64)
    if not np.all(np.isfinite(t)):
        return False
    if param in (PARAM_MC_ETA, PARAM_LNMC_ETA_LND):
        if param == PARAM_MC_ETA and t[0] <= 0:
            return False
        if not (0.0 < t[1] <= 0.25):
            return False
    elif param == PARAM_MC_Q:
        if t[0] <= 0 or t[1] <= 0:
            return False
    elif param == PARAM_M1M2:
        if t[0] <= 0 or t[1] <= 0:
            return False
    if abs(t[2]) > 1 or abs(t[3]) > 1:
        return False
    if param != PARAM_LNMC_ETA_LND and t[4] <= 0:
        return False
    return True


def spin_combinations(s):
    chi1, chi2, eta, delta = s["chi1"], s["chi2"], s["eta"], s["delta"]
    chis = 0.5 * (chi1 + chi2)
    chia = 0.5 * (chi1 - chi2)
    chi_eff = chis + delta * chia                       # (m1 chi1 + m2 chi2) / M
    chi_pn = chi_eff - 38.0 * eta / 113.0 * (chi1 + chi2)
    return chis, chia, chi_eff, chi_pn


# ====================================================================================
# coefficient fits (Sec. 3.1: 19 parameters x 11 fit terms = 209 coefficients)
# ====================================================================================

def fit_basis(eta, chi_pn):
    x = chi_pn - 1.0
    return [1.0, eta, x, x * eta, x * eta**2, x**2, x**2 * eta, x**2 * eta**2,
            x**3, x**3 * eta, x**3 * eta**2]


def fit_parameters(lam, eta, chi_pn):
    """Lambda_i(eta, chi_PN) = sum_k lam[i][k] B_k; returns a dict keyed by parameter name."""
    lam = np.asarray(lam).reshape(19, 11)
    b = fit_basis(eta, chi_pn)
    out = {}
    for i, name in enumerate(LAMBDA_NAMES):
        acc = 0.0
        for k in range(11):
            acc = acc + lam[i, k] * b[k]
        out[name] = acc
    return out


# ====================================================================================
# final state and ring-down (stand-ins: the model's own fits are not available)
# ====================================================================================

def final_spin(s):
    """Final dimensionless spin, aligned-spin fit of Barausse & Rezzolla (2009)."""
    m1 = s["M"] * (1.0 + s["delta"]) / 2.0
    m2 = s["M"] * (1.0 - s["delta"]) / 2.0
    eta = s["eta"]
    a_tilde = (m1**2 * s["chi1"] + m2**2 * s["chi2"]) / (m1**2 + m2**2)
    s4, s5, t0, t2, t3 = -0.1229, 0.4537, -2.8904, -3.5171, 2.5763
    return (a_tilde + s4 * a_tilde**2 * eta + s5 * a_tilde * eta**2 + t0 * a_tilde * eta
            + 2.0 * math.sqrt(3.0) * eta + t2 * eta**2 + t3 * eta**3)


def radiated_energy(s, chi_eff):
    """Radiated energy in units of M (stand-in: test-mass ISCO term + eta^2 correction)."""
    eta = s["eta"]
    return eta * (1.0 - 2.0 * math.sqrt(2.0) / 3.0) + eta**2 * (0.55 + 0.5 * chi_eff)


def ringdown_frequencies(a_f, e_rad):
    """(f_RD, f_damp) in units of 1/M from the l=m=2, n=0 quasi-normal-mode fit of
    Berti, Cardoso & Will (2006): M_f omega_R = f1 + f2 (1-a)^f3, Q = q1 + q2 (1-a)^q3,
    omega_I = omega_R / (2Q); M_f = M (1 - E_rad)."""
    omega_r = 1.5251 - 1.1568 * (1.0 - a_f) ** 0.1292
    qual = 0.7000 + 1.4187 * (1.0 - a_f) ** (-0.4990)
    omega_i = omega_r / (2.0 * qual)
    scale = 1.0 / (2.0 * math.pi * (1.0 - e_rad))
    return omega_r * scale, omega_i * scale


# ====================================================================================
# post-Newtonian coefficients (aligned spins)
# ====================================================================================

def taylorf2_phase_coefficients(eta, delta, chis, chia):
    """phi_k and log-coefficients phi_kl of Phi_TF2 = 3/(128 eta) sum_k (phi_k + phi_kl ln v) v^(k-5)."""
    pi = math.pi
    phi = [0.0] * 8
    phil = [0.0] * 8
    phi[0] = 1.0
    phi[2] = 3715.0 / 756.0 + 55.0 * eta / 9.0
    phi[3] = (-16.0 * pi + 113.0 / 3.0 * delta * chia + (113.0 / 3.0 - 76.0 * eta / 3.0) * chis)
    phi[4] = (15293365.0 / 508032.0 + 27145.0 * eta / 504.0 + 3085.0 * eta**2 / 72.0
              + (-405.0 / 8.0 + 200.0 * eta) * chia**2 - 405.0 / 4.0 * delta * chia * chis
              + (-405.0 / 8.0 + 5.0 * eta / 2.0) * chis**2)
    p5 = (38645.0 * pi / 756.0 - 65.0 * pi * eta / 9.0
          + delta * (-732985.0 / 2268.0 - 140.0 * eta / 9.0) * chia
          + (-732985.0 / 2268.0 + 24260.0 * eta / 81.0 + 340.0 * eta**2 / 9.0) * chis)
    phi[5] = p5                      # 2.5PN term multiplies (1 + 3 ln v)
    phil[5] = 3.0 * p5
    phi[6] = (11583231236531.0 / 4694215680.0 - 6848.0 * EULER_GAMMA / 21.0 - 640.0 * pi**2 / 3.0
              + (-15737765635.0 / 3048192.0 + 2255.0 * pi**2 / 12.0) * eta
              + 76055.0 * eta**2 / 1728.0 - 127825.0 * eta**3 / 1296.0
              - 6848.0 / 21.0 * math.log(4.0)
              + pi * delta * 2270.0 / 3.0 * chia + pi * (2270.0 / 3.0 - 520.0 * eta) * chis
              + (75515.0 / 144.0 - 8225.0 * eta / 18.0) * delta * chia * chis
              + (75515.0 / 288.0 - 263245.0 * eta / 252.0 - 480.0 * eta**2) * chia**2
              + (75515.0 / 288.0 - 232415.0 * eta / 504.0 + 1255.0 * eta**2 / 9.0) * chis**2)
    phil[6] = -6848.0 / 21.0         # from -6848/21 ln(4 v)
    phi[7] = (77096675.0 * pi / 254016.0 + 378515.0 * pi * eta / 1512.0 - 74045.0 * pi * eta**2 / 756.0
              + delta * (-25150083775.0 / 3048192.0 + 26804935.0 * eta / 6048.0 - 1985.0 * eta**2 / 48.0) * chia
              + (-25150083775.0 / 3048192.0 + 10566655595.0 * eta / 762048.0
                 - 1042165.0 * eta**2 / 3024.0 + 5345.0 * eta**3 / 36.0) * chis)
    return phi, phil


def pn_amplitude_coefficients(eta, delta, chis, chia):
    """A_i of the PN amplitude ratio sum_i A_i (pi Mf)^(i/3), i = 0..6 (A_0 = 1, A_1 = 0)."""
    pi = math.pi
    a = [0.0] * 7
    a[0] = 1.0
    a[2] = -323.0 / 224.0 + 451.0 * eta / 168.0
    a[3] = 27.0 / 8.0 * delta * chia + (27.0 / 8.0 - 11.0 * eta / 6.0) * chis
    a[4] = (-27312085.0 / 8128512.0 - 1975055.0 * eta / 338688.0 + 105271.0 * eta**2 / 24192.0
            + (-81.0 / 32.0 + 8.0 * eta) * chia**2 - 81.0 / 16.0 * delta * chia * chis
            + (-81.0 / 32.0 + 17.0 * eta / 8.0) * chis**2)
    a[5] = (-85.0 * pi / 64.0 + 85.0 * pi * eta / 16.0
            + delta * (285197.0 / 16128.0 - 1579.0 * eta / 4032.0) * chia
            + (285197.0 / 16128.0 - 15211.0 * eta / 1008.0 + 2351.0 * eta**2 / 4032.0) * chis)
    a[6] = (-177520268561.0 / 8583708672.0
            + (545384828789.0 / 5007163392.0 - 205.0 * pi**2 / 48.0) * eta
            - 3248849057.0 * eta**2 / 178827264.0 + 34473079.0 * eta**3 / 6386688.0
            + (1614569.0 / 64512.0 - 1873643.0 * eta / 16128.0 + 2167.0 * eta**2 / 42.0) * chia**2
            + (31.0 * pi / 12.0 - 7.0 * pi * eta / 3.0) * chis
            + (1614569.0 / 64512.0 - 61391.0 * eta / 1344.0 + 57451.0 * eta**2 / 4032.0) * chis**2
            + delta * chia * (31.0 * pi / 12.0 + (1614569.0 / 32256.0 - 165961.0 * eta / 2688.0) * chis))
    return a


# ====================================================================================
# the model on an array of dimensionless frequencies Mf
# ====================================================================================

class Model:
    """All per-source quantities of the model; `phase(mf)` / `amplitude_ratio(mf)` evaluate it.

    The inputs may be complex-step perturbed: every operation below is analytic and every
    branch decision looks at real parts only.
    """

    def __init__(self, theta, param, lam, f_ref):
        s = source(theta, param)
        self.s = s
        eta, delta = s["eta"], s["delta"]
        chis, chia, chi_eff, chi_pn = spin_combinations(s)
        self.eta = eta
        self.M = s["M"]
        self.Ms = s["M"] * T_SUN
        p = fit_parameters(lam, eta, chi_pn)
        self.p = p
        self.phi, self.phil = taylorf2_phase_coefficients(eta, delta, chis, chia)
        self.amp_pn = pn_amplitude_coefficients(eta, delta, chis, chia)
        a_f = final_spin(s)
        e_rad = radiated_energy(s, chi_eff)
        self.f_rd, self.f_damp = ringdown_frequencies(a_f, e_rad)

        # ---- amplitude: peak frequency of the merger-ringdown Lorentzian (O4 reading)
        g2, g3 = p["gamma2"], p["gamma3"]
        if np.real(g2) <= 1.0:
            x = g3 * self.f_damp * ((1.0 - g2**2) ** 0.5 - 1.0) / g2
        else:
            x = -g3 * self.f_damp / g2
        self.f_peak = self.f_rd + x

        # ---- phase join frequencies
        self.f_p1 = F_PHASE_JOIN
        self.f_p2 = 0.5 * self.f_rd
        self.f_a1 = F_AMP_JOIN
        self.valid = (np.real(self.f_peak) > F_AMP_JOIN) and (np.real(self.f_p2) > F_PHASE_JOIN)

        # ---- C1 phase connection (Sec. 3.1: continuous in the first derivative)
        f1 = self.f_p1
        self.c2_int = self.dphi_ins(f1) - self.dphi_int_raw(f1)
        self.c1_int = self.phi_ins(f1) - self.phi_int_raw(f1) - self.c2_int * f1
        f2 = self.f_p2
        self.c2_mrd = self.dphi_int(f2) - self.dphi_mrd_raw(f2)
        self.c1_mrd = self.phi_int(f2) - self.phi_mrd_raw(f2) - self.c2_mrd * f2

        # ---- intermediate amplitude: quartic through 5 conditions
        fa1, fa3 = self.f_a1, self.f_peak
        fa2 = 0.5 * (fa1 + fa3)
        rows = [[1.0, fa1, fa1**2, fa1**3, fa1**4],
                [0.0, 1.0, 2.0 * fa1, 3.0 * fa1**2, 4.0 * fa1**3],
                [1.0, fa2, fa2**2, fa2**3, fa2**4],
                [1.0, fa3, fa3**2, fa3**3, fa3**4],
                [0.0, 1.0, 2.0 * fa3, 3.0 * fa3**2, 4.0 * fa3**3]]
        rhs = [self.amp_ins(fa1), self.damp_ins(fa1), p["v2"], self.amp_mrd(fa3), self.damp_mrd(fa3)]
        dtype = np.result_type(*[np.asarray(v) for r in rows for v in r], *[np.asarray(v) for v in rhs])
        self.delta_int = np.linalg.solve(np.array(rows, dtype=dtype), np.array(rhs, dtype=dtype))

        # ---- time and phase alignment (O10 reading): t0 = Phi'_MRD(f_peak), reference at f_ref
        self.t0 = self.dphi_mrd(self.f_peak)
        self.mf_ref = self.Ms * f_ref
        self.phi_ref = self.phase_raw(np.array([self.mf_ref]))[0]

        # ---- overall amplitude: face-on, optimally oriented Newtonian SPA prefactor (O5 reading)
        self.amp0 = (math.sqrt(5.0 / 24.0) * math.pi ** (-2.0 / 3.0)
                     * (s["Mc"] * T_SUN) ** (5.0 / 6.0) * C_SI / (s["D"] * MPC_M))

    # ---------------- phase pieces (f = Mf) -------------------------------------------
    def phi_ins(self, f):
        v = (math.pi * f) ** (1.0 / 3.0)
        lv = np.log(v)
        acc = 0.0
        for k in range(8):
            acc = acc + (self.phi[k] + self.phil[k] * lv) * v ** (k - 5)
        tf2 = 3.0 / (128.0 * self.eta) * acc
        p = self.p
        pseudo = (p["sigma1"] * f + 0.75 * p["sigma2"] * f ** (4.0 / 3.0)
                  + 0.6 * p["sigma3"] * f ** (5.0 / 3.0) + 0.5 * p["sigma4"] * f**2) / self.eta
        return tf2 + pseudo

    def dphi_ins(self, f):
        v = (math.pi * f) ** (1.0 / 3.0)
        lv = np.log(v)
        acc = 0.0
        for k in range(8):
            n = k - 5
            acc = acc + (n * (self.phi[k] + self.phil[k] * lv) + self.phil[k]) * v ** (n - 3)
        dtf2 = 3.0 / (128.0 * self.eta) * (math.pi / 3.0) * acc
        p = self.p
        dpseudo = (p["sigma1"] + p["sigma2"] * f ** (1.0 / 3.0) + p["sigma3"] * f ** (2.0 / 3.0)
                   + p["sigma4"] * f) / self.eta
        return dtf2 + dpseudo

    def phi_int_raw(self, f):
        p = self.p
        return (p["beta1"] * f + p["beta2"] * np.log(f) - p["beta3"] / (3.0 * f**3)) / self.eta

    def dphi_int_raw(self, f):
        p = self.p
        return (p["beta1"] + p["beta2"] / f + p["beta3"] / f**4) / self.eta

    def phi_int(self, f):
        return self.phi_int_raw(f) + self.c1_int + self.c2_int * f

    def dphi_int(self, f):
        return self.dphi_int_raw(f) + self.c2_int

    def phi_mrd_raw(self, f):
        p = self.p
        return (p["alpha1"] * f - p["alpha2"] / f + 4.0 / 3.0 * p["alpha3"] * f**0.75
                + p["alpha4"] * np.arctan((f - p["alpha5"] * self.f_rd) / self.f_damp)) / self.eta

    def dphi_mrd_raw(self, f):
        p = self.p
        fd = self.f_damp
        return (p["alpha1"] + p["alpha2"] / f**2 + p["alpha3"] * f ** (-0.25)
                + p["alpha4"] * fd / (fd**2 + (f - p["alpha5"] * self.f_rd) ** 2)) / self.eta

    def phi_mrd(self, f):
        return self.phi_mrd_raw(f) + self.c1_mrd + self.c2_mrd * f

    def dphi_mrd(self, f):
        return self.dphi_mrd_raw(f) + self.c2_mrd

    def phase_raw(self, mf):
        """Piecewise phase before alignment: inspiral / intermediate / merger-ringdown."""
        mf = np.asarray(mf)
        re = np.real(mf)
        out = np.zeros(mf.shape, dtype=np.result_type(mf, np.asarray(self.c1_mrd)))
        i1 = re < self.f_p1
        i3 = re >= np.real(self.f_p2)
        i2 = ~(i1 | i3)
        if np.any(i1):
            out[i1] = self.phi_ins(mf[i1])
        if np.any(i2):
            out[i2] = self.phi_int(mf[i2])
        if np.any(i3):
            out[i3] = self.phi_mrd(mf[i3])
        return out

    # ---------------- amplitude pieces (ratio to the Newtonian amplitude) ------------
    def amp_ins(self, f):
        acc = 0.0
        for i in range(7):
            acc = acc + self.amp_pn[i] * (math.pi * f) ** (i / 3.0)
        p = self.p
        return acc + p["rho1"] * f ** (7.0 / 3.0) + p["rho2"] * f ** (8.0 / 3.0) + p["rho3"] * f**3

    def damp_ins(self, f):
        acc = 0.0
        for i in range(1, 7):
            acc = acc + self.amp_pn[i] * (i / 3.0) * math.pi ** (i / 3.0) * f ** (i / 3.0 - 1.0)
        p = self.p
        return (acc + 7.0 / 3.0 * p["rho1"] * f ** (4.0 / 3.0) + 8.0 / 3.0 * p["rho2"] * f ** (5.0 / 3.0)
                + 3.0 * p["rho3"] * f**2)

    def amp_mrd(self, f):
        p = self.p
        g = p["gamma3"] * self.f_damp
        x = f - self.f_rd
        return p["gamma1"] * g / (x**2 + g**2) * np.exp(-p["gamma2"] * x / g)

    def damp_mrd(self, f):
        p = self.p
        g = p["gamma3"] * self.f_damp
        x = f - self.f_rd
        return self.amp_mrd(f) * (-2.0 * x / (x**2 + g**2) - p["gamma2"] / g)

    def amp_int(self, f):
        d = self.delta_int
        return d[0] + d[1] * f + d[2] * f**2 + d[3] * f**3 + d[4] * f**4

    def amplitude_ratio(self, mf):
        mf = np.asarray(mf)
        re = np.real(mf)
        out = np.zeros(mf.shape, dtype=np.result_type(mf, np.asarray(self.delta_int[0])))
        i1 = re < self.f_a1
        i3 = re >= np.real(self.f_peak)
        i2 = ~(i1 | i3)
        if np.any(i1):
            out[i1] = self.amp_ins(mf[i1])
        if np.any(i2):
            out[i2] = self.amp_int(mf[i2])
        if np.any(i3):
            out[i3] = self.amp_mrd(mf[i3])
        return out

    # ---------------- on a physical frequency grid -----------------------------------
    def amp_phase(self, f, active):
        """Amplitude A(f) and phase Psi(f) on the active bins (physical f in Hz)."""
        s = self.s
        fa = f[active]
        mf = self.Ms * fa
        phase = (self.phase_raw(mf) - self.t0 * (mf - self.mf_ref) - self.phi_ref
                 + 2.0 * math.pi * fa * s["tc"] - 2.0 * s["phic"])
        amp = self.amp0 * fa ** (-7.0 / 6.0) * self.amplitude_ratio(mf)
        return amp, phase


def grid_freqs(grid):
    f0, df, n, f_min, f_ref = grid
    return f0 + np.arange(int(n), dtype=np.float64) * df


def active_mask(theta, param, grid):
    """Bins that carry signal: f >= f_min and M f <= 0.2."""
    f = grid_freqs(grid)
    s = source(np.asarray(theta, dtype=np.float64), param)
    ms = float(np.real(s["M"])) * T_SUN
    return (f >= grid[3]) & (ms * f <= F_CUT)


def amp_phase(theta, param, lam, grid, active=None):
    """(A, Psi, active) on the grid; A and Psi only on active bins."""
    if active is None:
        active = active_mask(theta, param, grid)
    model = Model(theta, param, lam, grid[4])
    if not model.valid:
        raise ValueError("model transition frequencies out of order for this source")
    amp, phase = model.amp_phase(grid_freqs(grid), active)
    return amp, phase, active


def waveform(theta, param, lam, grid, active=None):
    """Complex strain h_k = A_k exp(-i Psi_k) on the grid (zero on inactive bins)."""
    theta = np.asarray(theta, dtype=np.float64)
    h = np.zeros(int(grid[2]), dtype=np.complex128)
    if not domain_ok(theta, param):
        h[:] = np.nan
        return h
    amp, phase, act = amp_phase(theta, param, lam, grid, active)
    h[act] = amp * np.exp(-1j * phase)
    return h


def waveforms(thetas, param, lam, grid):
    return np.stack([waveform(t, param, lam, grid) for t in thetas])


# ====================================================================================
# inner products, likelihood, Fisher (Eq. 1, Eq. 8)
# ====================================================================================

def inner(a, b, inv_psd, df):
    """(a|b) = 4 df Re sum_k conj(a_k) b_k / S_k, summed with exact rounding (math.fsum)."""
    terms = (np.conj(a) * b).real * inv_psd
    return 4.0 * df * math.fsum(terms.tolist())


def overlaps(theta, param, lam, grid, streams, inv_psd):
    """Complex overlaps of one template with several data streams (Eq. 1 before taking the real
    part): O_s = 4 df sum_k conj(h_k) d_s,k / S_k, real and imaginary parts each summed with
    exact rounding; also returns (h|h).  Re O_s = (h|d_s) and |O_s| is the overlap maximised
    over a constant phase shift."""
    h = waveform(theta, param, lam, grid)
    df = grid[1]
    out = np.zeros(len(streams), dtype=np.complex128)
    for i, d in enumerate(streams):
        terms = np.conj(h) * np.asarray(d) * inv_psd
        out[i] = 4.0 * df * complex(math.fsum(terms.real.tolist()), math.fsum(terms.imag.tolist()))
    return out, inner(h, h, inv_psd, df)


def loglike(theta, param, lam, grid, data, inv_psd):
    """Gaussian log-likelihood up to the theta-independent -(d|d)/2: (d|h) - (h|h)/2."""
    h = waveform(theta, param, lam, grid)
    df = grid[1]
    return inner(data, h, inv_psd, df) - 0.5 * inner(h, h, inv_psd, df)


def _cs_step(x):
    return 1e-20 * max(1.0, abs(float(x)))


def amp_phase_derivatives(theta, param, lam, grid, active=None):
    """d ln A / d theta_p and d Psi / d theta_p on the active bins by complex-step
    differentiation (Im f(x + i h) / h), p = 0..6.  Returns (A, Psi, dlnA[7], dPsi[7], active)."""
    theta = np.asarray(theta, dtype=np.float64)
    amp, phase, act = amp_phase(theta, param, lam, grid, active)
    dlna = np.zeros((7, amp.size))
    dpsi = np.zeros((7, amp.size))
    for p in range(7):
        hstep = _cs_step(theta[p])
        tp = theta.astype(np.complex128)
        tp[p] += 1j * hstep
        a_c, ph_c, _ = amp_phase(tp, param, lam, grid, act)
        dlna[p] = np.imag(a_c) / hstep / amp
        dpsi[p] = np.imag(ph_c) / hstep
    return amp, phase, dlna, dpsi, act


def loglike_grad(theta, param, lam, grid, data, inv_psd):
    """d lnL / d theta (7) by complex-step through the real amplitude/phase form of lnL."""
    theta = np.asarray(theta, dtype=np.float64)
    act = active_mask(theta, param, grid)
    df = grid[1]
    dr, di, w = data.real[act], data.imag[act], inv_psd[act]
    g = np.zeros(7)
    for p in range(7):
        hstep = _cs_step(theta[p])
        tp = theta.astype(np.complex128)
        tp[p] += 1j * hstep
        a_c, ph_c, _ = amp_phase(tp, param, lam, grid, act)
        hr = a_c * np.cos(ph_c)
        hi = -a_c * np.sin(ph_c)
        lnl = 4.0 * df * np.sum(w * (dr * hr + di * hi)) - 0.5 * 4.0 * df * np.sum(w * a_c * a_c)
        g[p] = np.imag(lnl) / hstep
    return g


def fisher(theta, param, lam, grid, inv_psd):
    """F_pq = (d_p h | d_q h) with d_p h = h (d_p ln A - i d_p Psi)  (Eq. 8, one detector)."""
    amp, phase, dlna, dpsi, act = amp_phase_derivatives(theta, param, lam, grid)
    h = amp * np.exp(-1j * phase)
    dh = h[None, :] * (dlna - 1j * dpsi)
    w = inv_psd[act]
    df = grid[1]
    F = np.zeros((7, 7))
    for p in range(7):
        for q in range(7):
            F[p, q] = inner(dh[p], dh[q], w, df)
    return F


# ====================================================================================
# match and mismatch (Eqs. 3-4) and the gradient over the 209 coefficients
# ====================================================================================

def overlap_series(h1, h2, w):
    """z_j = sum_k w_k conj(h1_k) h2_k exp(+2 pi i k j / N), j = 0..N-1 (inverse DFT, unnormalised)."""
    n = len(h1)
    return np.fft.ifft(w * np.conj(h1) * h2) * n


def overlap_series_bruteforce(h1, h2, w):
    n = len(h1)
    k = np.arange(n)
    x = w * np.conj(h1) * h2
    return np.array([np.sum(x * np.exp(2j * math.pi * k * j / n)) for j in range(n)])


def match(h1, h2, w):
    """(m, lag j*, |z| top-two gap).  m = max_j |z_j| / sqrt((h1|h1)(h2|h2)); ties -> lowest j."""
    z = overlap_series(h1, h2, w)
    az = np.abs(z)
    j = int(np.argmax(az))          # numpy returns the first (lowest) index on ties
    a = math.fsum((w * np.abs(h1) ** 2).tolist())
    b = math.fsum((w * np.abs(h2) ** 2).tolist())
    srt = np.sort(az)
    gap = (srt[-1] - srt[-2]) / srt[-1] if len(srt) > 1 and srt[-1] > 0 else 1.0
    return az[j] / math.sqrt(a * b), j, gap


def mismatch(theta, param, lam, grid, target, w):
    h = waveform(theta, param, lam, grid)
    m, j, gap = match(h, target, w)
    return 1.0 - m, j, gap


def mismatch_grad_lambda(theta, param, lam, grid, target, w):
    """(mismatch, lag, gap, d mismatch / d lambda[209]).

    The maximising lag j* is held fixed (the derivative of a maximum over a discrete set is
    the derivative at its arg-max); the modulus |z_j*| is the maximum over the phase.  The
    mismatch at that lag is written in the real amplitude/phase of h1 and differentiated
    by complex step in each of the 209 coefficients.
    """
    theta = np.asarray(theta, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64).reshape(-1)
    mm, j, gap = mismatch(theta, param, lam, grid, target, w)
    act = active_mask(theta, param, grid)
    n = int(grid[2])
    k = np.arange(n)[act]
    x = w[act] * target[act] * np.exp(2j * math.pi * k * j / n)      # conj(h1) multiplies this
    xr, xi = x.real, x.imag
    b = math.fsum((w * np.abs(target) ** 2).tolist())
    grad = np.zeros(lam.size)
    for i in range(lam.size):
        hstep = _cs_step(lam[i])
        lp = lam.astype(np.complex128)
        lp[i] += 1j * hstep
        a_c, ph_c, _ = amp_phase(theta, param, lp, grid, act)
        c, s = np.cos(ph_c), np.sin(ph_c)
        # conj(h1) = A (cos Psi + i sin Psi)
        zr = np.sum(a_c * (c * xr - s * xi))
        zi = np.sum(a_c * (c * xi + s * xr))
        aa = np.sum(w[act] * a_c * a_c)
        mm_c = 1.0 - (zr * zr + zi * zi) ** 0.5 / (aa * b) ** 0.5
        grad[i] = np.imag(mm_c) / hstep
    return mm, j, gap, grad


def fit_lambda_step(thetas, param, lam, grid, targets, w, alpha):
    """One step of the coefficient fit of Sec. 3.1: the loss is the mean mismatch over the
    targets (Eq. 7) and the step is lambda - alpha * dL/dlambda (Eq. 6).  Returns (the updated
    coefficients, the mismatches [nt] and the summed gradient [209] at the coefficients given)."""
    lam = np.asarray(lam, dtype=np.float64).reshape(-1)
    mms = []
    gsum = np.zeros(lam.size)
    for th, tg in zip(thetas, targets):
        mm, _, _, g = mismatch_grad_lambda(th, param, lam, grid, tg, w)
        mms.append(mm)
        gsum += g
    return lam - alpha * (gsum / len(mms)), np.array(mms), gsum
