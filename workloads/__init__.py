"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds parameter sets and random draws only.  It contains none of the
method's arithmetic (no constitutive law, no discretisation, no solver step), so
that the CPU oracle and the HIP path can both take their inputs from here without
sharing any computation.

Random numbers the method draws (the KL coefficients xi_j, which the paper's
Karhunen-Loeve expansion takes as i.i.d. standard normals, Section 3 eq. KLexp)
come from numpy's PCG64 seeded by SeedSequence([workload id, level, sample]),
so that the fine and the coarse solve of one MLMC pair receive the same draw
(the paper's requirement that both levels of a correction use the same random
input, Section 5.1 eq. SMC).
"""
from __future__ import annotations

import numpy as np

# Gardner closure for the infiltration workloads (not in the paper, which uses
# van Genuchten-Mualem; the exponential Gardner law is the standard mild
# alternative and is what the benchmark workloads fix):
#   K = Ks*exp(a*h), theta = theta_r + (theta_s-theta_r)*exp(a*h) for h < 0.
GARDNER_INFILTRATION = dict(
    model="gardner",
    theta_r=0.05,
    theta_s=0.5,
    gardner_a=1.0,
    h_top=0.0,
    h_bottom=-10.0,
    h_init=-10.0,
    dt=0.01,
    n_steps=10,
)

# Lognormal Ks field: KL expansion of sigma^2 * exp(-sqrt(2) r / lam), which is
# the paper's Matern form at nu = 1/2 (Section 3 eq. nonIsotropic), truncated at
# 64 terms, mean log 0.
KS_FIELD = dict(sigma2=1.0, corr_len=0.3, log_mean=0.0, scale=1.0, n_modes=64)

# Multigrid / Picard settings of the throughput workloads: one V(2,2) cycle per
# modified-Picard step, Picard stopped when ||dp||_inf < 1e-8.
SOLVER = dict(
    cycle="V", nu1=2, nu2=2, cycles_per_picard=1, eps_picard=1e-8, eps_mg=1e-5,
    max_picard=100, coarsest_n=4,
)

# Small plain-MC workload: 32x32 grid, 16 samples, FP64.
PLAIN_MC_32 = dict(workload_id=0, n=32, n_samples=16)

# Batched MLMC workload: five levels, samples per level (a level >= 1 sample is
# a fine/coarse pair sharing one draw).
MLMC_5LEVEL = dict(workload_id=1, grids=(16, 32, 64, 128, 256),
                   samples=(4096, 1024, 256, 64, 16))

# Working set for the smoother roofline (larger than the 256 MB last-level cache).
SMOOTHER_ROOF = dict(workload_id=9, n=512, n_samples=64)

# van Genuchten-Mualem workload with three random fields and parametric
# continuation (Section 2.1 eqs. Sw, sc_van, Krw; Section 3; Section 5.2), on the
# problem every MLMC experiment of Section 6 uses: the infiltration problem of
# eq. travellingwave (p0 = -0.4 (1 - exp(-80 z)), p = -0.4 on top, 0.1 at the bottom,
# no flux on the sides) with the baseline conductivity Ks_bl = 0.2:
#   Ks    = 0.2 exp(G_K),             G_K a KL field of sigma^2 = 1.5;
#   alpha = exp(mu_a + s_a G_a),      mean 2;
#   n     = 1 + exp(mu_n + s_n G_n),  mean 1.6;
# every G a unit-variance KL field of the exponential kernel with correlation
# length 0.2, 128 terms, independent draws per field.  The spreads of alpha and
# n - 1 match the standard deviations of the paper's uniform perturbations
# (+-0.2 and +-0.05) with lognormal laws.  Continuation: level l of L + 1 solves
# with n shifted by (L - l) * 0.1 (milder on coarse levels); the coarse member of
# a level-l pair uses level l - 1's shift, as the fine member of pair l - 1 does.
# Time grid: 50 steps of dt = 0.005 (T = 0.25; Section 6 integrates to T = 0.2).
VG_SA2 = 0.003328
VG_SN2 = 0.002312
VG_KS_BASELINE = 0.2
VG_FIELDS = dict(
    corr_len=0.2, n_modes=128,
    marginals=((0.0, float(np.log(VG_KS_BASELINE)), float(np.sqrt(1.5))),        # Ks
               (0.0, float(np.log(2.0) - VG_SA2 / 2), float(np.sqrt(VG_SA2))),    # alpha
               (1.0, float(np.log(0.6) - VG_SN2 / 2), float(np.sqrt(VG_SN2)))),   # n
)
VG_INFILTRATION = dict(
    model="vg",
    theta_r=0.05,
    theta_s=0.5,
    h_top=-0.4,
    h_bottom=0.1,
    h_init=-0.4,
    init_rate=80.0,
    dt=0.005,
    n_steps=50,
)
MLMC_VG = dict(workload_id=2, grids=(32, 64, 128, 256, 512), samples=(2048, 512, 128, 32, 8),
               n_shift_grad=0.1)

# Robustness sweep of Section 4.3: the infiltration problem of eq. travellingwave
# (p0 = -0.4 (1 - exp(-80 z)), p = -0.4 on top, 0.1 at the bottom, no flux on the
# sides), van Genuchten-Mualem with theta_s = 0.5, theta_r = 0.05 and constant alpha,
# n per sample from Table alpha_n (20 x 20 pairs), Ks = 0.2 exp(Z) with Z the KL field
# of the Matern covariance Phi_1 = (1.0, 0.2, 0.2, 1) of Table Matern (64 modes),
# 64 samples per pair; W(2,2) cycles to eps_MG = 1e-5, eps_PI = 1e-5, at most 50
# Picard iterations per step; T = 0.1 reached with 7 steps of dt = 1/64 (h = 1/32).
SWEEP_ALPHA = (0.2, 0.4, 0.6, 0.8, 1.0, 1.2, 1.4, 1.6, 1.8, 2.0, 2.2, 2.4, 2.6, 2.8, 3.0, 3.2, 3.4, 3.6, 3.8, 4.0)
SWEEP_N = (1.1, 1.2, 1.3, 1.4, 1.5, 1.6, 1.7, 1.8, 1.9, 2.0, 2.2, 2.4, 2.6, 2.8, 3.0, 3.2, 3.4, 3.6, 3.8, 4.0)
MATERN_PHI1 = (1.0, 0.2, 0.2, 1.0)
MATERN_PHI2 = (0.5, 0.1, 0.01, 1.0)
TRAVELLING_WAVE = dict(model="vg", theta_r=0.05, theta_s=0.5, h_top=-0.4, h_bottom=0.1, h_init=-0.4,
                       init_rate=80.0, dt=1.0 / 64.0, n_steps=7, ks_baseline=0.2)
SWEEP = dict(workload_id=4, n=32, samples_per_pair=64, n_modes=64, eps=1e-5, eps_mg=1e-5, max_picard=50)
SWEEP_T_FINAL = 0.1

# Adaptive PC_MLMC (Algorithm 1) on the van Genuchten workload above: six levels 32^2 ..
# 1024^2 with n shifted by (L - l) * 0.1 on level l, 100 steps of dt = 0.0025 (the same
# T = 0.25 as MLMC_VG), RMSE target 1e-3 (sampling tolerance and the eq. discErr bias
# estimate), warm-up pairs per level.
PC_MLMC_VG = dict(workload_id=5, grids=(32, 64, 128, 256, 512, 1024), warmup=(64, 32, 16, 8, 4, 4),
                  n_shift_grad=0.1, n_steps_full=100, dt_full=0.0025, eps_full=1e-3)

# Adjoint sensitivities: the Gardner problem on 128 x 128 with 20 steps, Ks = exp(G) from a
# 100-term KL expansion of the same covariance as KS_FIELD, 1024 samples; the quantity is
# the time-integrated bottom outflux and its gradient in the 100 KL coefficients, with the
# forward pressure head checkpointed every 5 steps.
ADJOINT_128 = dict(workload_id=3, n=128, n_samples=1024, n_modes=100, n_steps=20, ckpt_every=5)


def xi_draws(workload_id: int, level: int, sample_ids, n_fields: int, n_modes: int) -> np.ndarray:
    """Standard-normal KL coefficients, shape [len(sample_ids)][n_fields][n_modes], float64."""
    sample_ids = list(sample_ids)
    out = np.empty((len(sample_ids), n_fields, n_modes), dtype=np.float64)
    for k, i in enumerate(sample_ids):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([workload_id, level, int(i)])))
        out[k] = rng.standard_normal((n_fields, n_modes))
    return out


def uniform_array(seed, shape, lo=0.0, hi=1.0) -> np.ndarray:
    """Seeded uniform float64 array (kernel-level test inputs)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(np.atleast_1d(seed)))))
    return rng.uniform(lo, hi, size=shape)


def normal_array(seed, shape) -> np.ndarray:
    """Seeded standard-normal float64 array (kernel-level test inputs)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(np.atleast_1d(seed)))))
    return rng.standard_normal(size=shape)
