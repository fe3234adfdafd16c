"""Write closed_forms.json: Dirichlet Laplacian eigenvalues in closed form.

The 1D Dirichlet second-difference matrix tridiag(-1, 2, -1) of size s has
eigenvalues 4 sin^2(i pi / (2(s+1))), i = 1..s; the 2D 5-point and 3D 7-point
Laplacians are Kronecker sums, so their eigenvalues are sums of these.  These
values pin the oracle (they are not produced by it).
"""
import json
import os

import numpy as np


def main():
    t32 = 4.0 * np.sin(np.arange(1, 33) * np.pi / 66) ** 2
    e2 = np.sort((t32[:, None] + t32[None, :]).ravel())[:6]
    t64 = 4.0 * np.sin(np.arange(1, 65) * np.pi / 130) ** 2
    e3 = np.sort((t64[:, None, None] + t64[None, :, None] + t64[None, None, :]).ravel())[:33]
    out = {
        "laplace2d_32": {"eigs": e2.tolist(), "norm2": float(8 * np.sin(32 * np.pi / 66) ** 2),
                         "note": "lambda_{ij} = 4 sin^2(i pi/66) + 4 sin^2(j pi/66); lambda_2 = lambda_3"},
        "laplace3d_64": {"eigs": e3[[0, 15, 16, 31, 32]].tolist(), "index": [1, 16, 17, 32, 33],
                         "note": "sum over three axes of 4 sin^2(i pi/130); lambda_16 = lambda_17"},
    }
    with open(os.path.join(os.path.dirname(__file__), "closed_forms.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
