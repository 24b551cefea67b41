"""Shared builders for GPU tests: workloads -> msv Plan, oracle references."""
from __future__ import annotations

import numpy as np

from oracle import assemble as oasm
from oracle import discretize as odisc
from oracle import modal as omodal
from oracle import solve as osolve
from workloads import geometry, incident, rules

RULES = rules.load_rules()


def sphere8_curve():
    return geometry.sphere(8)


def oracle_setup(curve, k0, eps1, M, L, mu1=1.0):
    sup = odisc.support_points(curve, *RULES)
    k1 = k0 * np.sqrt(complex(eps1 * mu1))
    if k1.imag < 0:
        k1 = -k1
    kp = omega_params = omodal.KernelParams(k0, k1, M, L, float(curve.r.max()))
    return sup, kp


def oracle_table(curve, sup, kp, rows=None):
    return omodal.tabulate(curve, sup, kp, rows=rows)


def oracle_matrix(curve, sup, tab, m, k0, k1, eps1, mu1=1.0, rows=None):
    w = geometry.gl_weights(curve)
    return oasm.assemble_mode(curve, sup, tab, m, k0, k1, k0, 1.0, 1.0, eps1, mu1, w, rows=rows)


def normwise_table_error(got, ref):
    """max over (type, target, source) of ||got - ref||_inf,m / ||ref||_inf,m."""
    diff = np.max(np.abs(got - ref), axis=0)
    scale = np.max(np.abs(ref), axis=0)
    ok = scale > 0
    err = np.zeros_like(scale)
    err[ok] = diff[ok] / scale[ok]
    zero_ref_bad = np.max(diff[~ok]) if np.any(~ok) else 0.0
    return float(err.max()), float(zero_ref_bad)
