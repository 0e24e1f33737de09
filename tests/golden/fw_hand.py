"""Writes fw_hand.json: Algorithm 1 (Section 2.3) worked by hand on the
smallest case, D = 2 and d = 1, evaluated in 50-digit decimal arithmetic.

With d = 1 the projections are rows a, b of length 2 and the loss of
Problem leanvec_efficient reduces to scalars and 2-vectors (K_Q, K_X
symmetric):

    f(a, b)  = (a K_Q a^T)(b K_X b^T) + tr(K_Q K_X) - 2 (a K_Q).(b K_X)
    df/da    = 2 (b K_X b^T) a K_Q - 2 (b K_X) K_Q
    df/db    = 2 (a K_Q a^T) b K_X - 2 (a K_Q) K_X

(Eq. leanvec_gradients for a 1 x D block).  The linear step over the unit
spectral-norm ball of 1 x 2 matrices is S = C / ||C||_2 (the SVD of a row
is its norm times its direction).  One iteration t, as Algorithm 1 orders
it: gamma = 1/(t+1)^alpha; the A-step from the gradient at (A^(t), B^(t));
the B-step from the gradient at (A^(t+1), B^(t)); and the early stop when
|f(A^(t+1), B^(t+1)) - f(A^(t), B^(t))| / f(A^(t), B^(t)) <= tol.

This file uses no code of the oracle or of the library: it evaluates the
formulas above, so the stored trace pins the oracle's and the library's
update order, step schedule and stop rule independently of both.
"""
import json
import os
from decimal import Decimal as Dc, getcontext

getcontext().prec = 50
KQ = [[Dc(3), Dc(1)], [Dc(1), Dc(4)]]
KX = [[Dc(11), Dc(3)], [Dc(3), Dc(45)]]
ALPHA = Dc("0.5")
A0, B0 = [Dc(1), Dc(0)], [Dc(0), Dc(1)]
T = 6


def row_times(v, K):
    return [v[0] * K[0][0] + v[1] * K[1][0], v[0] * K[0][1] + v[1] * K[1][1]]


def dot(u, v):
    return u[0] * v[0] + u[1] * v[1]


TR = sum(KQ[i][j] * KX[j][i] for i in range(2) for j in range(2))


def f(a, b):
    aK, bK = row_times(a, KQ), row_times(b, KX)
    return dot(aK, a) * dot(bK, b) + TR - 2 * dot(aK, bK)


def grad_a(a, b):
    aK, bK = row_times(a, KQ), row_times(b, KX)
    bKK = row_times(bK, KQ)
    return [2 * dot(bK, b) * aK[i] - 2 * bKK[i] for i in range(2)]


def grad_b(a, b):
    aK, bK = row_times(a, KQ), row_times(b, KX)
    aKK = row_times(aK, KX)
    return [2 * dot(aK, a) * bK[i] - 2 * aKK[i] for i in range(2)]


def unit(c):
    n = (c[0] ** 2 + c[1] ** 2).sqrt()
    return [c[0] / n, c[1] / n]


def trace():
    a, b = list(A0), list(B0)
    out = [dict(t=0, A=a, B=b, f=f(a, b))]
    for t in range(T):
        g = 1 / (Dc(t + 1) ** ALPHA)
        CA = [-x for x in grad_a(a, b)]
        SA = unit(CA)
        gap_a = dot([SA[i] - a[i] for i in range(2)], CA)
        a = [(1 - g) * a[i] + g * SA[i] for i in range(2)]
        CB = [-x for x in grad_b(a, b)]          # at (A^(t+1), B^(t))
        SB = unit(CB)
        gap_b = dot([SB[i] - b[i] for i in range(2)], CB)
        b = [(1 - g) * b[i] + g * SB[i] for i in range(2)]
        out.append(dict(t=t + 1, gamma=g, S_A=SA, S_B=SB, gap_A=gap_a, gap_B=gap_b, A=a, B=b,
                        f=f(a, b)))
    return out


def main():
    tr = trace()
    fl = [float(h["f"]) for h in tr]
    ratio = [float(abs(tr[t + 1]["f"] - tr[t]["f"]) / tr[t]["f"]) for t in range(T)]
    # tolerances at which the printed denominator f(A^(t), B^(t)) and the
    # other reading, f(A^(t+1), B^(t+1)), stop at different iterations
    stops = []
    for tol in (0.18, 0.05):
        it = next(t + 1 for t in range(T) if ratio[t] <= tol)
        stops.append({"tol": tol, "iters": it})
    fx = lambda v: [float(x) for x in v]  # noqa: E731
    doc = {
        "source": "Section 2.3, Algorithm 1 (Frank-Wolfe BCD), Eq. leanvec_gradients, Problem "
                  "leanvec_efficient (trace form); stop rule of Section 2.3",
        "derivation": __doc__.strip(),
        "KQ": [[float(x) for x in r] for r in KQ], "KX": [[float(x) for x in r] for r in KX],
        "m": 1, "n": 1, "D": 2, "d": 1, "alpha": float(ALPHA),
        "A0": fx(A0), "B0": fx(B0),
        "iterations": [{"t": h["t"], "A": fx(h["A"]), "B": fx(h["B"]), "f": float(h["f"]),
                        **({"gamma": float(h["gamma"]), "S_A": fx(h["S_A"]), "S_B": fx(h["S_B"]),
                            "gap_A": float(h["gap_A"]), "gap_B": float(h["gap_B"])}
                           if h["t"] else {})} for h in tr],
        "f": fl,
        "relative_change": ratio,
        "stops": stops,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fw_hand.json")
    with open(path, "w") as fh:
        json.dump(doc, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
