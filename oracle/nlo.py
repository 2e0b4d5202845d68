"""Integrated counterterms and the virtual correction -- ORACLE, TEST
INFRASTRUCTURE ONLY (the same rules as the rest of oracle/: only tests/, the
smoke check and the benchmark's CPU-baseline leg use it).

The paper's NLO cross section is Born + virtual + real (the section on
next-to-leading order corrections); the FKS subtraction makes the real
emission locally finite, and what it subtracts is added back, integrated in
d = 4 - 2 eps dimensions, where its poles cancel those of the virtual.  For a
Born with exactly two massless coloured partons of one flavour (e+e- -> u
ubar) every piece is proportional to the Born, and this module writes the
finite remainder out.

Counterterms (the reading of the kernels: always subtract, xi_c = xi_max = 1,
delta = 2, sector functions S_ij = (1/d_ij) / sum 1/d).  In the sector of
gluon i and quark j, with xi = x_i, y = cos(i, j) and D = 2 - xi (1 - y),
the three-body energy fractions are x_j = 2 (1 - xi) / D,
1 - x_j = xi (1 + y) / D, 1 - x_k = (1 - xi) xi (1 - y) / D, and the exact d-
dimensional phase space (orientations integrated)
    dPhi_3 = Phi_2 s / (16 pi^2) (4 pi / s)^eps / Gamma(1 - eps)
             [(1-x_1)(1-x_2)(1-x_3)]^(-eps) dx_1 dx_2
becomes, per unit Born, K(eps) xi^(-1-2eps) (1-y)^(-1-eps) G(xi, y) dxi dy with
    K = (alpha_s C_F / 2 pi) (4 pi mu^2 / s)^eps / Gamma(1 - eps),
    G = f [(1-xi)^2 (1+y) / D^2]^(-eps) 2 (1-xi) / D^2,
    f = xi^2 (1-y) |M_R|^2 S_ij / (B 2 C_F g^2 / s)   (finite at both limits).
At eps -> 0, G is the kernels' j g_R (the phase-space factor j = s E_j /
(64 pi^3 Ebar_j (1 - xi (1-y)/2)) times g_R), so subtracting G at xi = 0 and
y = 1 is exactly the density the device integrates.  What it subtracts is
  soft:      int dxi xi^(-1-2eps) int dy (1-y)^(-1-eps) [G(0,y) - G(0,1)]
             with G(0, y) = 2 ((1+y)/4)^(-eps) (eikonal x S^soft = 4);
  collinear: int dy (1-y)^(-1-eps) int dxi xi^(-1-2eps) [G(xi,1) - G(0,1)]
             with G(xi, 1) = [(1-eps) xi^2 + 2 (1-xi)] ((1-xi)^2 / 2)^(-eps)
             (the d-dimensional P_qq(z = 1 - xi) = C_F [(1+z^2)/(1-z) - eps (1-z)]);
  double:    G(0, 1) int dxi xi^(-1-2eps) int dy (1-y)^(-1-eps), G(0,1) = 2^(1+eps).
With int_0^1 xi^(-1-2eps) = -1/(2 eps), int_-1^1 (1-y)^(-1-eps) = -2^(-eps)/eps and
Beta functions for the rest, per sector
  soft = -zeta_2,  collinear = 3/(2 eps) + 13/2 - 4 zeta_2,  double = 1/eps^2,
so the two sectors give K B [2/eps^2 + 3/eps + 13 - 10 zeta_2] + O(eps).

Virtual: the one-loop quark form factor at timelike q^2 = s,
  V = B (alpha_s C_F / 2 pi) c_Gamma (4 pi mu^2 / s)^eps [-2/eps^2 - 3/eps - 8 + pi^2],
  c_Gamma = Gamma(1+eps) Gamma(1-eps)^2 / Gamma(1-2eps) = 1/Gamma(1-eps) + O(eps^3)
(the pi^2 is Re (-1)^(-eps) times the double pole).  The poles cancel, and
  (V + integrated counterterms)_finite = B (alpha_s C_F / 2 pi) (5 - 2 pi^2 / 3),
independent of mu.  Together with the integrated subtracted real emission,
sigma_NLO = sigma_B (1 + alpha_s / pi) (the textbook e+e- -> hadrons result),
which the tests check."""
import math

ZETA2 = math.pi ** 2 / 6
CF = 4.0 / 3.0


def vi_coefficient(alpha_s):
    """(V + integrated counterterms)_finite / B for e+e- -> q qbar"""
    return alpha_s * CF / (2 * math.pi) * (5.0 - 4.0 * ZETA2)


def counterterm_laurent():
    """Per-sector coefficients (eps^-2, eps^-1, eps^0) of soft + collinear +
    double, in units of K B (see the module text)"""
    return 1.0, 1.5, 6.5 - 5.0 * ZETA2


def virtual_integrated(orc, mom):
    """e+e- -> u ubar Born points mom [4][4][n] -> (B, (V + I)_finite) per event, GeV^-2"""
    b = orc.me2("ee_uu", mom)
    return b, b * vi_coefficient(orc._params[1] if orc._params else 0.118)
