"""Small helpers shared by the tests: Minkowski products, boosts, couplings.

Plain textbook formulae, used to check results; none of the method's
arithmetic lives here."""
import math

import numpy as np

ALPHA = 1.0 / 132.507
ALPHA_S = 0.118
M_TOP = 173.0
E2 = 4 * math.pi * ALPHA
G2 = 4 * math.pi * ALPHA_S


def mdot(a, b):
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]


def boost_matrix(beta):
    """Pure Lorentz boost with velocity vector beta (3,)."""
    b2 = float(np.dot(beta, beta))
    g = 1.0 / math.sqrt(1.0 - b2)
    L = np.eye(4)
    L[0, 0] = g
    L[0, 1:] = L[1:, 0] = g * beta
    L[1:, 1:] += (g - 1.0) * np.outer(beta, beta) / b2
    return L


def rotation_matrix(axis, angle):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    R = np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * K @ K
    L = np.eye(4)
    L[1:, 1:] = R
    return L


def transform(mom, L):
    """mom [npart, 4, n] -> L applied to every four-vector."""
    return np.einsum('ij,pjn->pin', L, mom)
