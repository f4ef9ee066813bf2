"""Writes the hand-derived golden fixtures of this folder.

Each value is a closed form worked out by hand from the paper's equations for a
tiny case (the derivation is stored next to it); this script only evaluates
those closed forms with the math module.  It calls neither the oracle nor the
HIP library.  Run: python tests/golden/make_golden.py
"""
import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def fixtures():
    e1, e2, e4 = math.exp(-1.0), math.exp(-2.0), math.exp(-4.0)
    a = 1 / math.sqrt(2) - 0.05
    return {
        "linear_two_steps.json": {
            "cite": "Sec. II-D real split and time index n = 2t + l - 1; eqn:apsm with W = 1; "
                    "eqn:beta; Fact 1 with wG = 0",
            "derivation": "M=1, K=1, one pilot r = 0.6+0.8i, b = (1+i)/sqrt2, wL = 0.5, wG = 0, W = 1, "
                          "mu = 1, eps = 0.05. r1 = [0.6, 0.8], r2 = [0.8, -0.6], both unit norm and "
                          "orthogonal. Step 0: f0 = 0, e = 0, e - Re b = -1/sqrt2 < -eps, kappa(r1,r1) = "
                          "wL*1 = 0.5, beta = (1/sqrt2 - eps)/0.5, w += beta*wL*r1 = (1/sqrt2 - eps) r1. "
                          "Step 1: e = w.r2 = 0 by orthogonality, same beta, w += (1/sqrt2 - eps) r2. "
                          "Final w = (1/sqrt2 - eps)(r1 + r2) = (1/sqrt2 - eps)[1.4, 0.2]; g(r) = f(r1) "
                          "+ i f(r2) = (1/sqrt2 - eps)(1 + i).",
            "params": {"sigma2": 0.5, "eps": 0.05, "mu": 1.0, "window": 1, "w_lin": 0.5,
                       "w_gauss": 0.0, "dict_cap": None},
            "rx_pilot": [[0.6, 0.8]], "sym_pilot": [[[1 / math.sqrt(2), 1 / math.sqrt(2)]]],
            "expected_w": [[a * 1.4, a * 0.2]],
            "expected_g_at_pilot": [[a, a]],
        },
        "gauss_two_steps.json": {
            "cite": "Sec. II-A Gaussian kernel; eqn:apsm with W = 1; eqn:beta with eps = 0; Gaussian "
                    "dictionary of Sec. II-D; FIFO cap reading",
            "derivation": "M=1, K=1, r = 1+0i so r1 = [1,0], r2 = [0,-1]; b = 1+1i; wL = 0, wG = 1, "
                          "sigma2 = 0.5, eps = 0, W = 1, mu = 1. Step 0: e = 0, kappa(r1,r1) = wG = 1, "
                          "beta = 1, alpha(r1) = 1. Step 1 uncapped: e = exp(-||r1-r2||^2/(2*0.5)) = "
                          "exp(-2), beta = 1 - exp(-2) = alpha(r2). f(r1) = 1 + (1 - e^-2) e^-2, f(r2) = "
                          "e^-2 + 1 - e^-2 = 1. With a cap of one entry, r1 is evicted before step 1 "
                          "predicts, so e = 0, alpha(r2) = 1 and f = kappa_G(r2, .): f(r1) = e^-2, f(r2) = 1.",
            "params": {"sigma2": 0.5, "eps": 0.0, "mu": 1.0, "window": 1, "w_lin": 0.0, "w_gauss": 1.0},
            "rx_pilot": [[1.0, 0.0]], "sym_pilot": [[[1.0, 1.0]]],
            "uncapped": {"dict_cap": None, "expected_alpha": [[1.0], [1 - e2]],
                         "expected_g_at_pilot": [[1 + e2 - e4, 1.0]]},
            "cap1": {"dict_cap": 1, "expected_alpha": [[1.0]], "expected_g_at_pilot": [[e2, 1.0]]},
        },
        "detect_two_entries.json": {
            "cite": "Sec. III-B detection f(r) = <f, kappa(r, .)>; Sec. II-D g(r) = f(r1) + i f(r2); "
                    "Sec. II-A kernels",
            "derivation": "M=1, K=1, w = [0.5, -0.25], dictionary d1 = [1,0], d2 = [0,1], alpha = "
                          "[0.3, -0.2], sigma2 = 1. At r = 0+1i: r1 = [0,1], r2 = [1,0]. f(r1) = -0.25 + "
                          "0.3 e^-1 - 0.2; f(r2) = 0.5 + 0.3 - 0.2 e^-1.",
            "sigma2": 1.0, "w": [[0.5, -0.25]], "dict": [[1.0, 0.0], [0.0, 1.0]],
            "alpha": [[0.3], [-0.2]], "rx": [[0.0, 1.0]],
            "expected_soft": [[[-0.45 + 0.3 * e1, 0.8 - 0.2 * e1]]],
        },
    }


if __name__ == "__main__":
    for name, fx in fixtures().items():
        with open(os.path.join(HERE, name), "w") as fh:
            json.dump(fx, fh, indent=1)
