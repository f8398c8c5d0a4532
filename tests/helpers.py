"""Shared test plumbing: workload -> Params, tolerance checks, oracle runs."""
import numpy as np

import workloads as W

KIND = {"coord": 1, "q6": 2, "coord_q6": 3}


def params_for(wl: dict, precision=None, hill_capacity=None, max_neighbors=64):
    from paper_2510_06873_amd import FP32, FP64, Params

    prec = {"fp32": FP32, "fp64": FP64}[precision or wl["precision"]]
    return Params(cv_kind=KIND[wl["cv"]], precision=prec, r_c=wl["r_c"], skin=wl["skin"],
                  taper=wl.get("taper", 0.2) or 0.2, cn_r0=wl.get("cn_r0", 2.5), bond_d0=wl.get("bond_d0", 0.7),
                  bond_w=wl.get("bond_w", 0.02), count_n0=wl.get("count_n0", 5.5), count_w=wl.get("count_w", 0.25),
                  sigma=wl["sigma"], w0=wl["w0"], gamma=wl["gamma"], kBT=wl["kBT"],
                  hill_capacity=hill_capacity or wl["hills"]["k"] + 16, max_neighbors=max_neighbors)


def oracle_cvs(orc, pos, box, wl, nl=None):
    """Oracle CV values and gradients for a workload's CV kind: (s[dims], [grads])."""
    nl = nl if nl is not None else orc.neighbors(pos, box, wl["r_c"] + wl["skin"])
    s, g = [], []
    if wl["cv"] in ("coord", "coord_q6"):
        s.append(orc.cn_forward(pos, box, nl, wl["cn_r0"], wl["r_c"]))
        g.append(orc.cn_gradient(pos, box, nl, wl["cn_r0"], wl["r_c"]))
    if wl["cv"] in ("q6", "coord_q6"):
        prm = orc.q6_params(wl["r_c"], wl["taper"], wl["bond_d0"], wl["bond_w"], wl["count_n0"], wl["count_w"])
        s.append(orc.q6_forward(pos, box, nl, prm)["s"])
        g.append(orc.q6_gradient(pos, box, nl, prm))
    return np.array(s), g, nl


def rel_force_err(F_gpu_bias, F_ref_bias):
    """max_i |dF_i| / max_i |F_ref_i|  (norm-wise over atoms)."""
    d = np.linalg.norm(np.asarray(F_gpu_bias, np.float64) - F_ref_bias, axis=1).max()
    return d / max(np.linalg.norm(F_ref_bias, axis=1).max(), 1e-300)


def structure(wl):
    return W.structure(wl["structure"])
