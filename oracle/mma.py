"""Oracle Method of Moving Asymptotes for one inequality constraint.  Test infrastructure
only (see oracle/__init__.py).

The paper solves eq. optprob with MMA (Sec. 5.1; Svanberg's method) and a move limit of
0.2 (Sec. 6.1); it does not state the method's remaining parameters.  Written from
Svanberg's description of MMA, with his standard choices:

* asymptotes: in the first two iterations L = x - 0.5 (xmax - xmin), U = x + 0.5 (xmax - xmin);
  later the distance of each asymptote to x grows by 1.2 where the last two steps of x_j
  had the same sign, shrinks by 0.7 where they alternated, and stays otherwise, kept
  within [0.01, 10] (xmax - xmin) of x;
* bounds of the subproblem: alpha = max(xmin, L + 0.1 (x - L), x - move),
  beta = min(xmax, U - 0.1 (U - x), x + move);
* convex separable approximations of the objective and of the constraint g <= 0 at x_k,
  h(x) = sum_j p_j / (U_j - x_j) + q_j / (x_j - L_j) + r, with
  p = (U - x)^2 (1.001 max(d, 0) + 0.001 max(-d, 0) + 1e-5),
  q = (x - L)^2 (0.001 max(d, 0) + 1.001 max(-d, 0) + 1e-5)  (d the derivative; the small
  terms keep every approximation strictly convex), and r such that h(x_k) = value.

The subproblem (minimise the objective's approximation subject to the constraint's, within
[alpha, beta]) is strictly convex and separable.  With one constraint its Lagrangian dual is
a concave function of a single multiplier lambda >= 0: for given lambda each x_j minimises
P_j / (U_j - x_j) + Q_j / (x_j - L_j) with P = p0 + lambda p1, Q = q0 + lambda q1, i.e.
x_j = (sqrt(P) L_j + sqrt(Q) U_j) / (sqrt(P) + sqrt(Q)) clipped to [alpha_j, beta_j], and the
dual's derivative is the constraint's approximation at x(lambda), non-increasing in lambda.
lambda = 0 if that is already feasible, else the root of the derivative, found by
bisection; if no point of [alpha, beta] satisfies the approximation, the limit lambda -> inf
(the point that reduces the constraint's approximation most).  (Svanberg's later formulation adds artificial variables that keep an
infeasible subproblem solvable; with one volume constraint and a start that satisfies it
they stay zero, and they are left out.)
"""

import numpy as np

ASY_INIT, ASY_INCR, ASY_DECR = 0.5, 1.2, 0.7
ALBEFA = 0.1
RAA0 = 1e-5


class MMA:
    def __init__(self, n, xmin=0.0, xmax=1.0, move=0.2):
        self.n, self.xmin, self.xmax, self.move = n, xmin, xmax, move
        self.k = 0
        self.xold1 = self.xold2 = None
        self.low = self.upp = None

    def _asymptotes(self, x):
        span = self.xmax - self.xmin
        if self.k <= 2:
            self.low = x - ASY_INIT * span
            self.upp = x + ASY_INIT * span
        else:
            sign = (x - self.xold1) * (self.xold1 - self.xold2)
            fac = np.where(sign > 0, ASY_INCR, np.where(sign < 0, ASY_DECR, 1.0))
            self.low = x - fac * (self.xold1 - self.low)
            self.upp = x + fac * (self.upp - self.xold1)
            self.low = np.clip(self.low, x - 10.0 * span, x - 0.01 * span)
            self.upp = np.clip(self.upp, x + 0.01 * span, x + 10.0 * span)

    @staticmethod
    def _pq(d, ux, xl):
        dp, dm = np.maximum(d, 0.0), np.maximum(-d, 0.0)
        return ux * ux * (1.001 * dp + 0.001 * dm + RAA0), xl * xl * (0.001 * dp + 1.001 * dm + RAA0)

    def subproblem(self, x, df, g, dg):
        """Data of the subproblem at x: (alpha, beta, p0, q0, p1, q1, b) with the constraint
        approximation written as sum_j p1/(U - x_j) + q1/(x_j - L) <= b."""
        alpha = np.maximum.reduce([np.full_like(x, self.xmin), self.low + ALBEFA * (x - self.low), x - self.move])
        beta = np.minimum.reduce([np.full_like(x, self.xmax), self.upp - ALBEFA * (self.upp - x), x + self.move])
        ux, xl = self.upp - x, x - self.low
        p0, q0 = self._pq(df, ux, xl)
        p1, q1 = self._pq(dg, ux, xl)
        b = np.sum(p1 / ux + q1 / xl) - g
        return alpha, beta, p0, q0, p1, q1, b

    def x_of(self, lam, alpha, beta, p0, q0, p1, q1):
        P, Q = p0 + lam * p1, q0 + lam * q1
        sp, sq = np.sqrt(P), np.sqrt(Q)
        return np.clip((sp * self.low + sq * self.upp) / (sp + sq), alpha, beta)

    def x_inf(self, alpha, beta, p1, q1):
        """Minimiser of the constraint's approximation alone over [alpha, beta] (lambda -> inf)."""
        sp, sq = np.sqrt(p1), np.sqrt(q1)
        return np.clip((sp * self.low + sq * self.upp) / (sp + sq), alpha, beta)

    def constraint(self, x, p1, q1, b):
        return np.sum(p1 / (self.upp - x) + q1 / (x - self.low)) - b

    def update(self, x, df, g, dg):
        """One MMA iteration from x with objective gradient df, constraint value g (the
        constraint is g <= 0) and gradient dg.  Returns (new x, lambda)."""
        x = np.asarray(x, dtype=float)
        self.k += 1
        self._asymptotes(x)
        alpha, beta, p0, q0, p1, q1, b = self.subproblem(x, df, g, dg)
        sub = (alpha, beta, p0, q0, p1, q1)
        if self.constraint(self.x_of(0.0, *sub), p1, q1, b) <= 0.0:
            lam = 0.0
            xnew = self.x_of(lam, *sub)
        elif self.constraint(self.x_inf(alpha, beta, p1, q1), p1, q1, b) > 0.0:
            # no point of the box satisfies the constraint's approximation (the move limit is
            # too tight): the limit lambda -> infinity, the point that reduces it most
            lam = np.inf
            xnew = self.x_inf(alpha, beta, p1, q1)
        else:
            lo, hi = 0.0, 1.0
            while self.constraint(self.x_of(hi, *sub), p1, q1, b) > 0.0:
                lo, hi = hi, 2.0 * hi
            for _ in range(400):
                mid = 0.5 * (lo + hi)
                if mid <= lo or mid >= hi:
                    break
                if self.constraint(self.x_of(mid, *sub), p1, q1, b) > 0.0:
                    lo = mid
                else:
                    hi = mid
            lam = hi
            xnew = self.x_of(lam, *sub)
        self.xold2 = self.xold1 if self.xold1 is not None else x.copy()
        self.xold1 = x.copy()
        self.last = dict(alpha=alpha, beta=beta, p0=p0, q0=q0, p1=p1, q1=q1, b=b, lam=lam)
        return xnew, lam
