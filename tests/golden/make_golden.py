"""Write the exact-arithmetic golden fixtures of tests/golden/.

The paper prints no worked numerical example, so the golden values are the
exact solutions of small rational UFTOC problems P(N) (Sec. 2), obtained by
solving their KKT system (Sec. 3) in rational arithmetic with
``oracle.exact`` only.  Run from the repository root:

    python tests/golden/make_golden.py
"""
import json
import os
import sys
from fractions import Fraction as Fr

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle import exact  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def tiny_problems():
    # n_x = 2, n_u = 1, N = 3: every term of P(N) nonzero, non-symmetric A,
    # cross term Qxw, affine a, constants c.
    p1 = dict(
        Qx=[[[2, Fr(1, 2)], [Fr(1, 2), 1]], [[1, 0], [0, 3]], [[Fr(3, 2), Fr(-1, 4)], [Fr(-1, 4), 2]]],
        Qw=[[[3]], [[Fr(5, 2)]], [[1]]],
        Qxw=[[[Fr(1, 4)], [0]], [[0], [Fr(-1, 2)]], [[Fr(1, 3)], [Fr(1, 5)]]],
        A=[[[1, Fr(1, 2)], [Fr(-1, 3), Fr(4, 5)]], [[Fr(9, 10), 0], [Fr(1, 4), Fr(7, 10)]],
           [[0, 1], [Fr(-1, 2), Fr(1, 2)]]],
        B=[[[1], [Fr(1, 2)]], [[0], [1]], [[Fr(2, 3)], [Fr(-1, 3)]]],
        a=[[Fr(1, 10), Fr(-1, 5)], [0, Fr(1, 2)], [Fr(-1, 4), 0]],
        lx=[[1, -1], [Fr(1, 2), 0], [0, Fr(3, 2)]],
        lw=[[Fr(-1, 2)], [1], [Fr(1, 4)]],
        c=[1, Fr(-1, 2), Fr(1, 3)],
        QxN=[[2, 1], [1, 2]], lN=[Fr(1, 2), -1], cN=Fr(3, 4),
        x0=[1, -2],
    )
    # scalar problem, N = 2, zero terminal (the MHE convention of Sec. 2)
    p2 = dict(
        Qx=[[[1]], [[2]]], Qw=[[[1]], [[Fr(1, 2)]]], Qxw=[[[0]], [[Fr(1, 4)]]],
        A=[[[Fr(1, 2)]], [[2]]], B=[[[1]], [[-1]]], a=[[1], [0]],
        lx=[[0], [1]], lw=[[1], [0]], c=[0, 0],
        QxN=[[0]], lN=[0], cN=0, x0=[3],
    )
    # n_x = 1, n_u = 2 (more inputs than states), N = 1
    p3 = dict(
        Qx=[[[1]]], Qw=[[[2, Fr(1, 2)], [Fr(1, 2), 1]]], Qxw=[[[Fr(1, 3), 0]]],
        A=[[[Fr(3, 2)]]], B=[[[1, -2]]], a=[[Fr(1, 2)]],
        lx=[[-1]], lw=[[0, 1]], c=[2],
        QxN=[[4]], lN=[1], cN=-1, x0=[Fr(-1, 2)],
    )
    return dict(tiny_n2_m1_N3=p1, scalar_N2_zero_terminal=p2, n1_m2_N1=p3)


def to_str(v):
    if isinstance(v, dict):
        return {k: to_str(e) for k, e in v.items()}
    if isinstance(v, list):
        return [to_str(e) for e in v]
    return str(Fr(v))


def main():
    out = {}
    for name, prob in tiny_problems().items():
        sol = exact.solve(prob)
        out[name] = dict(problem=to_str(prob), solution=to_str(sol))
    path = os.path.join(HERE, "tiny_exact.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print("wrote", path)


if __name__ == "__main__":
    main()
