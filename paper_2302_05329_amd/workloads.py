"""Seeded synthetic inputs shaped like the paper's workloads.

This module draws parameter points, builds frequency grids, evaluates the analytic
PSD stand-in and draws coloured Gaussian noise.  It is shared by the GPU path, the
tests and the CPU oracle's timing, and it deliberately contains none of the
waveform model's arithmetic: it only produces inputs.

Parameter rows are returned in the (m1, m2, chi1, chi2, D, tc, phic) layout
(masses in solar masses, D in Mpc, tc in s, phic in rad); `to_param` re-expresses
them in the other supported parameterisations.

The paper's data (detector PSD files, NR waveforms) are not available, so:
  * the PSD is the analytic zero-detuned high-power advanced-LIGO fit of Ajith (2011),
    standing in for the design curves the paper uses for Fisher forecasts and HMC
    (Sec. 3.2, Sec. 3.3);
  * noise follows the paper's Sec. 3.3 recipe: Gaussian, consistent with the PSD
    (real and imaginary parts i.i.d. N(0, S_n / (4 df)));
  * coefficient-fit targets (Sec. 3.1) are model waveforms built from a perturbed
    coefficient table instead of NR simulations.
"""
import os

import numpy as np

PARAM_MC_ETA = 0
PARAM_LNMC_ETA_LND = 1
PARAM_MC_Q = 2
PARAM_M1M2 = 3

# Solar-mass time GM_sun/c^3 in seconds (IAU 2015 nominal GM_sun); used only to lay out
# the mass-scaled grid of the coefficient-fit workload (Mf spacing fixed, Sec. 3.1).
_T_SUN_S = 1.3271244e20 / 299792458.0**3

_DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


def load_lambda(path=None):
    """The 19x11 coefficient table as a flat float64 array of 209 (row-major)."""
    if path is None:
        path = os.path.join(_DATA_DIR, "phenomd_lambda_placeholder.txt")
    rows = []
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(t) for t in line.split()])
    table = np.asarray(rows, dtype=np.float64)
    if table.shape != (19, 11):
        raise ValueError(f"coefficient table {path} has shape {table.shape}, want (19, 11)")
    return table.reshape(-1).copy()


def psd_aligo_zdhp_fit(f):
    """Analytic one-sided aLIGO zero-detuned high-power PSD fit (Ajith 2011), 1/Hz."""
    x = np.asarray(f, dtype=np.float64) / 215.0
    return 1e-49 * (x**-4.14 - 5.0 * x**-2 + 111.0 * (1.0 - x**2 + 0.5 * x**4) / (1.0 + 0.5 * x**2))


class Grid:
    """Uniform frequency grid f_k = f0 + k*df, k < n_bins.

    Bins with f_k < f_min carry no signal; f_ref is the physical frequency at which
    the phase is referenced.
    """

    def __init__(self, f0, df, n_bins, f_min=None, f_ref=20.0):
        self.f0 = float(f0)
        self.df = float(df)
        self.n_bins = int(n_bins)
        self.f_min = float(f0 if f_min is None else f_min)
        self.f_ref = float(f_ref)

    def freqs(self):
        k = np.arange(self.n_bins, dtype=np.float64)
        return self.f0 + k * self.df

    def as_tuple(self):
        return (self.f0, self.df, self.n_bins, self.f_min, self.f_ref)

    def __repr__(self):
        return (f"Grid(f0={self.f0}, df={self.df}, n_bins={self.n_bins}, "
                f"f_min={self.f_min}, f_ref={self.f_ref})")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def draw_masses(rng, n, lo=5.0, hi=50.0):
    a = rng.uniform(lo, hi, n)
    b = rng.uniform(lo, hi, n)
    return np.maximum(a, b), np.minimum(a, b)


def lambda_gamma2_above_one():
    """The placeholder table with the constant term of gamma2 raised by 0.35, so that
    1.1 < gamma2 < 1.2 over the configs' priors: the merger-ringdown amplitude then has no
    stationary point and the amplitude peak takes the other branch of its definition."""
    lam = load_lambda().reshape(19, 11).copy()
    lam[5, 0] += 0.35
    return lam.reshape(-1)


def draw_sources(n, seed, *, d_range=None, d_fixed=440.0, tc_range=None, phic_random=False,
                 chi_max=0.9):
    """n parameter rows (m1, m2, chi1, chi2, D, tc, phic) with the configs' priors."""
    rng = _rng(seed)
    m1, m2 = draw_masses(rng, n)
    chi1 = rng.uniform(-chi_max, chi_max, n)
    chi2 = rng.uniform(-chi_max, chi_max, n)
    if d_range is not None:
        dist = rng.uniform(d_range[0], d_range[1], n)
    else:
        dist = np.full(n, float(d_fixed))
    tc = rng.uniform(tc_range[0], tc_range[1], n) if tc_range is not None else np.zeros(n)
    phic = rng.uniform(0.0, 2.0 * np.pi, n) if phic_random else np.zeros(n)
    return np.stack([m1, m2, chi1, chi2, dist, tc, phic], axis=1)


def to_param(rows, param):
    """Re-express (m1, m2, ...) rows in another parameterisation (input preparation)."""
    rows = np.asarray(rows, dtype=np.float64)
    out = rows.copy()
    m1, m2 = rows[:, 0], rows[:, 1]
    mt = m1 + m2
    eta = m1 * m2 / mt**2
    mc = (m1 * m2) ** 0.6 / mt**0.2
    if param == PARAM_M1M2:
        return out
    if param == PARAM_MC_ETA:
        out[:, 0], out[:, 1] = mc, eta
    elif param == PARAM_LNMC_ETA_LND:
        out[:, 0], out[:, 1], out[:, 4] = np.log(mc), eta, np.log(rows[:, 4])
    elif param == PARAM_MC_Q:
        out[:, 0], out[:, 1] = mc, m2 / m1
    else:
        raise ValueError(f"unknown parameterisation {param}")
    return out


def complex_noise(psd, df, seed):
    """Gaussian noise consistent with a one-sided PSD: Re, Im i.i.d. N(0, S/(4 df))."""
    rng = _rng(seed)
    sigma = np.sqrt(np.asarray(psd) / (4.0 * df))
    n = len(sigma)
    return sigma * rng.standard_normal(n) + 1j * sigma * rng.standard_normal(n)


# ----------------------------------------------------------------------------------
# The five workloads.  Sizes are the full ones; `small=True` gives a shrunken copy
# with the same structure (for quick parity runs).
# ----------------------------------------------------------------------------------

def config1(n=1024, seed=1001):
    """Plain waveform evaluation: 20-1024 Hz, df = 0.25 Hz (4017 bins), D = 440 Mpc."""
    grid = Grid(20.0, 0.25, 4017, f_min=20.0, f_ref=20.0)
    theta = draw_sources(n, seed, d_fixed=440.0)
    return dict(name="C1 waveform_eval 1024x4017", theta=theta, grid=grid)


def config2(n=65536, seed=1002):
    """Batched fused log-likelihood: 20-2048 Hz, df = 0.125 Hz (16225 bins)."""
    grid = Grid(20.0, 0.125, 16225, f_min=20.0, f_ref=20.0)
    theta = draw_sources(n, seed, d_range=(100.0, 2000.0), tc_range=(-0.1, 0.1), phic_random=True)
    f = grid.freqs()
    psd = psd_aligo_zdhp_fit(f)
    data = complex_noise(psd, grid.df, seed)
    return dict(name="C2 loglike+grad 65536x16225", theta=theta, grid=grid, psd=psd,
                inv_psd=1.0 / psd, data=data)


def config3(n=16384, seed=1003):
    """7x7 Fisher matrices: 20-1024 Hz, df = 0.0625 Hz (16065 bins), config-1 priors."""
    grid = Grid(20.0, 0.0625, 16065, f_min=20.0, f_ref=20.0)
    theta = draw_sources(n, seed, d_fixed=440.0)
    psd = psd_aligo_zdhp_fit(grid.freqs())
    return dict(name="C3 fisher 16384x16065", theta=theta, grid=grid, psd=psd, inv_psd=1.0 / psd)


def config4(n=512, seed=1004, n_fft=65536, lam0=None, rel_sigma=0.01):
    """Mismatch gradient over the fit coefficients.

    Total mass fixed at 50 Msun, flat PSD, grid uniform in Mf from 0 to 0.2 with n_fft
    bins; bins below Mf = 2.5e-3 carry no signal (Sec. 3.1 and its footnote).  Targets
    share one perturbed table lam* = lam0 * (1 + rel_sigma * xi), xi ~ N(0, I).
    """
    rng = _rng(seed)
    a, b = draw_masses(rng, n)
    q = b / a
    mt = 50.0
    m1 = mt / (1.0 + q)
    m2 = mt - m1
    chi1 = rng.uniform(-0.9, 0.9, n)
    chi2 = rng.uniform(-0.9, 0.9, n)
    theta = np.stack([m1, m2, chi1, chi2, np.full(n, 440.0), np.zeros(n), np.zeros(n)], axis=1)
    ms = mt * _T_SUN_S
    df = 0.2 / (n_fft * ms)
    grid = Grid(0.0, df, n_fft, f_min=2.5e-3 / ms, f_ref=20.0)
    if lam0 is None:
        lam0 = load_lambda()
    xi = rng.standard_normal(lam0.shape)
    lam_star = lam0 * (1.0 + rel_sigma * xi)
    return dict(name="C4 mismatch_grad 512x65536", theta=theta, grid=grid,
                inv_psd=np.ones(n_fft), lam0=lam0, lam_star=lam_star)


def config5(seed=1005):
    """Learned-proposal sampling: one injection, 20-1024 Hz, df = 0.125 Hz (8033 bins)."""
    grid = Grid(20.0, 0.125, 8033, f_min=20.0, f_ref=20.0)
    mc, q = 30.0, 0.8
    eta = q / (1.0 + q) ** 2
    mt = mc * eta ** -0.6
    m1 = mt / (1.0 + q)
    m2 = mt - m1
    inj = np.array([m1, m2, 0.3, -0.2, 1.0, 0.0, 0.0])  # D set later for SNR 20
    psd = psd_aligo_zdhp_fit(grid.freqs())
    noise = complex_noise(psd, grid.df, seed)
    return dict(name="C5 flow-MH vs HMC 4096 chains x 8033", inj_unit_distance=inj, grid=grid,
                psd=psd, inv_psd=1.0 / psd, noise=noise, n_chains=4096, snr=20.0)


# Detector geometry in Earth-fixed Cartesian coordinates (metres; arm directions are unit
# vectors): the published site descriptions of LIGO Hanford (H1), LIGO Livingston (L1) and Virgo
# (V1), as compiled for the LIGO/Virgo analysis libraries (Althouse, Jones and Lazzarini,
# LIGO-P000006; the Virgo values from the same compilation).  Inputs only: vertex, x arm, y arm.
DETECTORS = {
    "H1": ((-2.16141492636e+06, -3.83469517889e+06, 4.60035022664e+06),
           (-0.22389266154, 0.79983062746, 0.55690487831),
           (-0.91397818574, 0.02609403989, -0.40492342125)),
    "L1": ((-7.42760447238e+04, -5.49628371971e+06, 3.22425701744e+06),
           (-0.95457412153, -0.14158077340, -0.26218911324),
           (0.29774156894, -0.48791033647, -0.82054461286)),
    "V1": ((4.54637409900e+06, 8.42989697626e+05, 4.37857696241e+06),
           (-0.70045821479, 0.20848948619, 0.68256166277),
           (-0.05379255368, -0.96908180549, 0.24080451708)),
}


def network_sources(n, seed, d_range=(100.0, 2000.0)):
    """Rows of 11 parameters for the detector network: the 7 of `draw_sources` (m1, m2, chi1, chi2,
    D, tc, phic) followed by inclination iota (cos iota uniform in [-1, 1]), polarisation psi
    (uniform in [0, pi)), right ascension alpha (uniform in [0, 2 pi)) and declination delta
    (sin delta uniform in [-1, 1]): isotropic orientation and sky position."""
    base = draw_sources(n, seed, d_range=d_range, tc_range=(-0.1, 0.1), phic_random=True)
    rng = _rng(seed + 50000)
    iota = np.arccos(rng.uniform(-1.0, 1.0, n))
    psi = rng.uniform(0.0, np.pi, n)
    alpha = rng.uniform(0.0, 2.0 * np.pi, n)
    delta = np.arcsin(rng.uniform(-1.0, 1.0, n))
    return np.concatenate([base, np.stack([iota, psi, alpha, delta], axis=1)], axis=1)


def network_config(n=65536, dets=("H1", "L1", "V1"), seed=1007, n_bins=16225, df=0.125, gmst=1.234):
    """Detector-network likelihood: C2's grid and source priors with isotropic orientation and sky
    position, one noise realisation per detector (analytic PSD stand-in for every site), and a
    fixed Greenwich sidereal angle gmst (rad) at the reference time."""
    grid = Grid(20.0, df, n_bins, f_min=20.0, f_ref=20.0)
    theta = network_sources(n, seed)
    psd = psd_aligo_zdhp_fit(grid.freqs())
    data = np.stack([complex_noise(psd, grid.df, seed + 10 * k) for k in range(len(dets))])
    return dict(name=f"network lnL+grad {n}x{n_bins}x{len(dets)}", theta=theta, grid=grid, dets=tuple(dets),
                geometry=[DETECTORS[d] for d in dets], psd=psd, inv_psd=np.stack([1.0 / psd] * len(dets)),
                data=data, gmst=gmst)


def fig1_sweep(n=10000, seed=1006):
    """Precision sweep shaped like the paper's Fig. 1 comparison: component masses uniform in
    (1, 100) Msun and aligned spins uniform in (-1, 1), D = 440 Mpc, on 32-1024 Hz with
    df = 0.0125 Hz (79361 bins), weighted by the analytic PSD stand-in (the paper uses a
    detector PSD from a catalogue release, not available here)."""
    rng = _rng(seed)
    m1 = rng.uniform(1.0, 100.0, n)
    m2 = rng.uniform(1.0, 100.0, n)
    chi = rng.uniform(-1.0, 1.0, (n, 2))
    theta = np.stack([m1, m2, chi[:, 0], chi[:, 1], np.full(n, 440.0), np.zeros(n), np.zeros(n)], axis=1)
    grid = Grid(32.0, 0.0125, 79361, f_min=32.0, f_ref=32.0)
    psd = psd_aligo_zdhp_fit(grid.freqs())
    return dict(name="Fig. 1 sweep 10000x79361", theta=theta, grid=grid, psd=psd, inv_psd=1.0 / psd)


def paper_timing_grid():
    """The paper's waveform-timing grid: 24-512 Hz, df = 0.2 Hz (2441 bins)."""
    return Grid(24.0, 0.2, 2441, f_min=24.0, f_ref=24.0)


# ----------------------------------------------------------------------------------
# Learned-proposal flow: random parameter vectors in the RealNVP layout (8 layers of
# W1[7][128] b1[128] W2[128][128] b2[128] W3[128][14] b3[14], then mu[7], isd[7]).
# ----------------------------------------------------------------------------------
FLOW_DIM, FLOW_HIDDEN, FLOW_OUT, FLOW_LAYERS = 7, 128, 14, 8


def flow_init_params(seed, mu=None, sd=None, out_scale=0.0, bias_scale=0.0):
    """float32 parameters: hidden weights ~ N(0, 1/fan_in), output weights ~ N(0, out_scale^2/128)
    (0 gives the identity map after standardisation, the usual start of training), biases
    ~ N(0, bias_scale^2); standardisation mu, isd = 1/sd."""
    rng = _rng(seed)
    d, h, o = FLOW_DIM, FLOW_HIDDEN, FLOW_OUT
    parts = []
    for _ in range(FLOW_LAYERS):
        parts += [rng.standard_normal(d * h) / np.sqrt(d), bias_scale * rng.standard_normal(h),
                  rng.standard_normal(h * h) / np.sqrt(h), bias_scale * rng.standard_normal(h),
                  out_scale * rng.standard_normal(h * o) / np.sqrt(h), bias_scale * rng.standard_normal(o)]
    mu = np.zeros(d) if mu is None else np.asarray(mu, dtype=np.float64)
    sd = np.ones(d) if sd is None else np.asarray(sd, dtype=np.float64)
    parts += [mu, 1.0 / sd]
    return np.concatenate(parts).astype(np.float32)


def correlated_gaussian(n, seed, dim=7, rho=0.45):
    """n draws of a dim-D Gaussian with unequal scales and a banded correlation (mean, cov, draws)."""
    rng = _rng(seed)
    mean = rng.uniform(-2.0, 2.0, dim)
    scale = np.exp(rng.uniform(-1.5, 1.0, dim))
    corr = np.eye(dim) + rho * (np.eye(dim, k=1) + np.eye(dim, k=-1))
    cov = corr * np.outer(scale, scale)
    x = rng.multivariate_normal(mean, cov, size=n)
    return mean, cov, x


def banana(n, seed, dim=7, b=0.5):
    """n draws of a curved ('banana') density: x1 += b (x0^2 - 1) on a standard Gaussian."""
    rng = _rng(seed)
    x = rng.standard_normal((n, dim))
    x[:, 1] += b * (x[:, 0] ** 2 - 1.0)
    return x
