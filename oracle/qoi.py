"""Scalar quantities of interest (oracle, FP64).

The paper's quantity of interest is the pressure field at the final time
(Section 5.1); the workloads here use scalar functionals of it:
  * mean effective saturation at the final time: (1/N) sum_c S_e(p_c(T)),
    S_e = (theta - theta_r)/(theta_s - theta_r);
  * time-integrated bottom outflux (accumulated by ``picard.solve``).
"""
from __future__ import annotations

import math

import numpy as np

from . import constitutive


def mean_saturation(problem, fields, p):
    se = constitutive.effective_saturation(problem, p, fields)
    return math.fsum(np.asarray(se, dtype=np.float64).ravel()) / se.size
