"""Closed forms of flat LambdaCDM used by the oracle's physics pins (test code only).

These are written from the mathematics, not from the oracle: the comoving distance and
the linear growth factor of a flat universe with matter and a cosmological constant
have hypergeometric closed forms,

    chi(a) = (c/H0) [x 2F1(1/2, 1/3; 4/3; -Om x^3/OL)] evaluated from x = 1 to x = 1/a, / sqrt(OL)
    D1(a)  = a 2F1(1/3, 1; 11/6; -OL a^3 / Om)          (D1 -> a deep in matter domination)

and in the Einstein-de Sitter limit (Om = 1) chi = 2 (c/H0)(1 - sqrt(a)), D1 = a.
"""
import math

from scipy import optimize, special

C_H0 = 299792.458 / 100.0          # c / H0 in Mpc/h


def chi_of_a(a, om):
    if om == 1.0:
        return 2.0 * C_H0 * (1.0 - math.sqrt(a))
    ol = 1.0 - om
    F = lambda x: x * special.hyp2f1(0.5, 1.0 / 3.0, 4.0 / 3.0, -om * x ** 3 / ol)
    return C_H0 * (F(1.0 / a) - F(1.0)) / math.sqrt(ol)


def a_of_chi(chi, om):
    if chi <= 0.0:
        return 1.0
    return optimize.brentq(lambda a: chi_of_a(a, om) - chi, 1e-3, 1.0, xtol=1e-15,
                           rtol=1e-15, maxiter=400)


def growth_D1(a, om):
    if om == 1.0:
        return a
    ol = 1.0 - om
    return a * special.hyp2f1(1.0 / 3.0, 1.0, 11.0 / 6.0, -ol * a ** 3 / om)
