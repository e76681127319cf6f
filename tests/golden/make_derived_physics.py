"""Write tests/golden/derived_physics.txt: closed-form and quadrature values of
the physics inputs the paper leaves unstated, computed here from their
textbook definitions with numpy and scipy only (no import of the oracle or of
the product package), so that the oracle's pins compare it with something
other than itself.

  alpha_s(t)   one-loop running, n_f = 5, alpha_s(M_Z^2) = 0.118 (the value the
               paper quotes with its jet-rate figure); App. A takes alpha_s at
               the emission's transverse momentum squared
  sigma_LO     e+e- -> (gamma, Z) -> q qbar, five massless flavours, summed over
               helicities and colours, integrated over the angle (App. B):
               sum_f 4 pi alpha^2 N_c / (3 s) [Q_f^2 - 2 Q_f v_e v_f chi_1
               + (a_e^2 + v_e^2)(a_f^2 + v_f^2) chi_2], in pb
  B/A          forward-backward over symmetric coefficient of A (1 + c^2) + B c:
               B = -4 Q_f a_e a_f chi_1 + 8 a_e a_f v_e v_f chi_2
  Delta        no-emission probability from t = s down to t_C of a q qbar start
               (two quark dipole ends with Q^2 = s), the Sudakov factor of App. A:
               exp(-2 int dt/t alpha_s(t)/(2 pi) int dz C_F [2/(1 - z(1 - y))
               - (1 + z)] (1 - y)), y = t/(s z (1 - z)) < 1 (Catani-Seymour
               final-final q -> q g kernel with its phase-space factor 1 - y)

Electroweak inputs: M_Z = 91.1876, Gamma_Z = 2.4952, alpha = 1/128.802,
sin^2 theta_W = 1 - (80.385/M_Z)^2.

Run from the repository root: python tests/golden/make_derived_physics.py
"""
import os
import sys

import numpy as np
from scipy import integrate

MZ, GZ, MW = 91.1876, 2.4952, 80.385
ALPHA, ASMZ, NC, CF = 1 / 128.802, 0.118, 3.0, 4.0 / 3.0
PB = 0.389379656e9  # GeV^-2 -> pb
SW2 = 1.0 - (MW / MZ) ** 2
A_E, V_E = -0.5, -0.5 + 2.0 * SW2
FLAVOURS = [(-1 / 3, -0.5), (2 / 3, 0.5), (-1 / 3, -0.5), (2 / 3, 0.5), (-1 / 3, -0.5)]  # (Q_f, T3_f): d u s c b

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "derived_physics.txt")


def alpha_s(t):
    b0 = (33.0 - 2.0 * 5) / (12.0 * np.pi)
    return ASMZ / (1.0 + ASMZ * b0 * np.log(t / MZ ** 2))


def chis(s):
    kappa = 1.0 / (4.0 * SW2 * (1.0 - SW2))
    den = (s - MZ ** 2) ** 2 + GZ ** 2 * MZ ** 2
    return kappa * s * (s - MZ ** 2) / den, kappa ** 2 * s ** 2 / den


def coefficients(qf, t3, s):
    af, vf = t3, t3 - 2.0 * qf * SW2
    c1, c2 = chis(s)
    A = qf ** 2 - 2.0 * qf * V_E * vf * c1 + (A_E ** 2 + V_E ** 2) * (af ** 2 + vf ** 2) * c2
    B = -4.0 * qf * A_E * af * c1 + 8.0 * A_E * af * V_E * vf * c2
    return A, B


def sigma_lo(ecm):
    s = ecm * ecm
    return sum(4 * np.pi * ALPHA ** 2 * NC / (3 * s) * coefficients(q, t3, s)[0] for q, t3 in FLAVOURS) * PB


def end_density(t, q2):
    """dP/d ln t of one quark end: alpha_s/(2 pi) int dz V (1 - y)."""
    if 4 * t >= q2:
        return 0.0
    r = np.sqrt(1 - 4 * t / q2)

    def f(z):
        y = t / (q2 * z * (1 - z))
        return CF * (2 / (1 - z * (1 - y)) - (1 + z)) * (1 - y)

    val, _ = integrate.quad(f, 0.5 * (1 - r), 0.5 * (1 + r), epsabs=0, epsrel=1e-11, limit=400)
    return alpha_s(t) / (2 * np.pi) * val


def sudakov(ecm, tc):
    s = ecm * ecm
    val, _ = integrate.quad(lambda lt: end_density(np.exp(lt), s), np.log(tc), np.log(s / 4), epsabs=0,
                            epsrel=1e-10, limit=400)
    return np.exp(-2 * val)


def lines():
    out = ["# Closed-form values under the readings of the paper's unstated physics inputs",
           "# (one-loop alpha_s with n_f = 5 and alpha_s(M_Z^2) = 0.118; LO e+e- -> q qbar with",
           "# M_Z = 91.1876, Gamma_Z = 2.4952, alpha = 1/128.802, sin^2 theta_W = 1 - (80.385/M_Z)^2;",
           "# Catani-Seymour final-final q -> q g kernel with the (1 - y) phase-space factor).",
           "# Written by tests/golden/make_derived_physics.py (numpy and scipy only, no oracle).",
           "#",
           "# alpha_s(t)  [App. A, Sudakov factor: alpha_s at p_T^2]"]
    for t in (0.25, 0.5, 1, 2, 4):
        out.append(f"alpha_s {t:g} {alpha_s(t):.6f}")
    out.append("# sigma_LO(sqrt s) in pb, five massless flavours  [App. B, differential cross-section]")
    for ecm in (10, 35, 91.2, 200, 500):
        out.append(f"sigma {ecm:g} {sigma_lo(ecm):.6g}")
    out.append("# forward-backward coefficient ratio B/A of A (1 + c^2) + B c at sqrt s = 91.2")
    for name, (q, t3) in (("ba_down", FLAVOURS[0]), ("ba_up", FLAVOURS[1])):
        A, B = coefficients(q, t3, 91.2 ** 2)
        out.append(f"{name} 91.2 {B / A:.5f}")
    out.append("# no-emission probability Delta(t_C, s) from a q qbar start (two quark ends)  [App. A, eq. Sudakov]")
    for ecm, tc in ((91.2, 1.0), (91.2, 0.25), (10, 1.0), (500, 0.25)):
        out.append(f"sudakov {ecm:g} {tc:g} {sudakov(ecm, tc):.5g}")
    return out


if __name__ == "__main__":
    text = "\n".join(lines()) + "\n"
    if "--check" in sys.argv:
        sys.exit(0 if open(OUT).read() == text else 1)
    open(OUT, "w").write(text)
    print(OUT)
