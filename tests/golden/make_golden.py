"""Writes the stored expected values under tests/golden/.

critical_line.json: Theorem (dynamics of F_1) (iv) of the paper (section 3.4):
for H = diag(lam_i, lam_j), lam_i < lam_j, starting on the ij-critical line at
r+ = (sqrt(lam_j/(lam_i+lam_j)), sqrt(lam_i/(lam_i+lam_j))) (unit norm), the
k-th residual of first-order CTA has norm rho_ij^k with
rho_ij = (lam_j - lam_i) / (lam_j + lam_i).  The values below are that closed
form, nothing else.
"""
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def critical_line():
    cases = []
    for li, lj, K in [(1.0, 3.0, 12), (2.0, 5.0, 10), (1.0, 100.0, 20), (0.25, 0.5, 8)]:
        rho = (lj - li) / (lj + li)
        cases.append({"lam_i": li, "lam_j": lj, "rho_ij": rho,
                      "expected_rel_res": [rho ** k for k in range(K + 1)]})
    return {"source": "Theorem on the dynamics of F_1, part (iv), section 3.4 (eqs. c-two, c-three)",
            "cases": cases}


if __name__ == "__main__":
    with open(os.path.join(HERE, "critical_line.json"), "w") as f:
        json.dump(critical_line(), f, indent=1)
