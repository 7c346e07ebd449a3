"""Derivation of ``restart_trace_1x1.json``: the restarted PDHG of Section 2.4.2
with the primal-weight update of Algorithm 4 on one 1 x 1 LP, worked in
60-digit decimal arithmetic.

It imports nothing from the solver or from the oracle: every step below is
written from the paper's definitions, so the stored trace pins the oracle's
restart rule from outside it.

The LP: min 3x  s.t.  x = 4,  x >= 0 (one "=" row, K = [1], u = +inf).
Its optimum is x* = 4, y* = 3 (lambda* = c - K^T y* = 0).

* Ruiz scaling (Algorithm 3) leaves K = [1] unchanged (every row and column
  norm is 1), and the power iteration (Algorithm 2) returns ||K|| = 1, so
  eta = 0.9 and omega_0 = ||c|| / ||q|| = 3/4 (Section 2.4.3).
* One step (Algorithm 1 in the sign-consistent form of Appendices C-D):
  x+ = proj_X(x - tau (c - K^T y)), xbar = 2x+ - x, y+ = y + sigma (q - K xbar)
  with tau = eta/omega, sigma = eta omega; the start is x = proj_X(0) = 0,
  y = 0.
* A check after every iteration (check period 1): the epoch average is the
  plain mean of the epoch's iterates; the candidate is the iterate when its
  KKT_omega is strictly smaller, else the average.
* KKT_omega(z) = sqrt(omega^2 pres^2 + dres^2 / omega^2 + gap^2) with
  pres = |x - 4|, lambda = proj_{R+}(3 - y) (x has only a lower bound),
  dres = |3 - y - lambda|, gap = |4y + 0 * lambda - 3x|.
* Restart when KKT(cand) <= 0.2 KKT(z0) (sufficient decay), or
  KKT(cand) <= 0.8 KKT(z0) and KKT(cand) > KKT(previous candidate) (necessary
  decay and no progress; no previous candidate at an epoch start), or the
  epoch's iterations exceed 0.36 of all iterations (long inner loop).
* On restart: Delta_x = |x_cand - x_0|, Delta_y = |y_cand - y_0| (distances
  from the epoch start); when both exceed 1e-6,
  omega <- exp(0.5 ln(Delta_y / Delta_x) + 0.5 ln omega); the new epoch starts
  at the candidate and its reference value is KKT_omega of the candidate at
  the new omega.
* Termination: relative KKT (Section 2.3.2) of the candidate, then of the
  other point, at most eps = 1e-6; rel-KKT = max(gap / (1 + |dobj| + |pobj|),
  pres / (1 + |q|), dres / (1 + |c|)).

Run ``python tests/golden/restart_1x1.py`` to rewrite the JSON file.
"""
import json
import os
from decimal import Decimal, getcontext

getcontext().prec = 60
D = Decimal

C, Q, L = D(3), D(4), D(0)
EPS = D("1e-6")


def terms(x, y):
    """pres, dres, gap, rel-KKT of (x, y) for the LP above (Section 2.3.2)."""
    pres = abs(x - Q)
    d = C - y
    lam = d if d > 0 else D(0)
    dres = abs(d - lam)
    pobj = C * x
    dobj = Q * y + (L * lam if lam > 0 else D(0))
    gap = abs(dobj - pobj)
    rel = max(gap / (1 + abs(dobj) + abs(pobj)), pres / (1 + abs(Q)), dres / (1 + abs(C)))
    return pres, dres, gap, rel


def kkt_w(t, w):
    pres, dres, gap, _ = t
    return (w * w * pres * pres + dres * dres / (w * w) + gap * gap).sqrt()


def derive():
    eta = D("0.9")
    omega = C / Q
    x, y = D(0), D(0)
    x0, y0 = x, y
    kkt0 = kkt_w(terms(x, y), omega)
    prev = None
    k_total = t_inner = 0
    sx = sy = D(0)
    recs = []
    while True:
        tau, sigma = eta / omega, eta * omega
        xn = max(x - tau * (C - y), L)
        y = y + sigma * (Q - (2 * xn - x))
        x = xn
        k_total += 1
        t_inner += 1
        sx += x
        sy += y
        xa, ya = sx / t_inner, sy / t_inner
        tc, ta = terms(x, y), terms(xa, ya)
        kc, ka = kkt_w(tc, omega), kkt_w(ta, omega)
        cand_avg = not (kc < ka)
        kcand, tcand = (ka, ta) if cand_avg else (kc, tc)
        rec = dict(iter=k_total, t_inner=t_inner, cand_avg=int(cand_avg), kkt_cand=kcand, kkt0=kkt0,
                   kkt_prev=prev, omega_before=omega, cand_pres=tcand[0], cand_dres=tcand[1],
                   cand_gap=tcand[2], rel_kkt_cur=tc[3], rel_kkt_avg=ta[3], restarted=0,
                   delta_x=D(0), delta_y=D(0))
        other = tc if cand_avg else ta
        if tcand[3] <= EPS or other[3] <= EPS:
            rec.update(stop=1, omega=omega, kkt0_next=kkt0, criteria=[])
            recs.append(rec)
            return recs
        suff = kcand <= D("0.2") * kkt0
        nec = kcand <= D("0.8") * kkt0 and prev is not None and kcand > prev
        art = D(t_inner) > D("0.36") * D(k_total)
        rec["criteria"] = [n for n, f in (("sufficient", suff), ("necessary", nec), ("artificial", art)) if f]
        if suff or nec or art:
            cx, cy = (xa, ya) if cand_avg else (x, y)
            dx, dy = abs(cx - x0), abs(cy - y0)
            if dx > EPS and dy > EPS:
                omega = ((dy / dx).ln() / 2 + omega.ln() / 2).exp()
            x, y = cx, cy
            x0, y0 = x, y
            kkt0 = kkt_w(tcand, omega)
            prev = None
            t_inner = 0
            sx = sy = D(0)
            rec.update(restarted=1, delta_x=dx, delta_y=dy)
        else:
            prev = kcand
        rec.update(stop=0, omega=omega, kkt0_next=kkt0)
        recs.append(rec)


def main():
    recs = derive()
    out = []
    for r in recs:
        o = {}
        for k, v in r.items():
            if isinstance(v, Decimal):
                o[k] = float(v)
            elif v is None:
                o[k] = "inf"
            else:
                o[k] = v
        out.append(o)
    doc = {
        "cite": "Section 2.4.2 (KKT_omega, candidate, three restart criteria with 0.2 / 0.8 / 0.36), "
                "Algorithm 4 (primal weight, read as Delta_y / Delta_x), Section 2.3.2 (termination)",
        "derivation": "restart_1x1.py beside this file: 60-digit decimal arithmetic from the paper's "
                      "definitions, no solver or oracle code",
        "lp": {"c": [3.0], "q": [4.0], "row_type": [1], "l": [0.0], "u": ["inf"], "K": [[1.0]]},
        "opts": {"check_every": 1, "eps": 1e-6, "ruiz_iters": 10, "eta": 0.9, "omega0": 0.75},
        "checks": out,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "restart_trace_1x1.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print(f"{len(out)} checks, {sum(r['restarted'] for r in out)} restarts -> {path}")


if __name__ == "__main__":
    main()
