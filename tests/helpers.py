"""Comparison metrics shared by the parity tests."""
import numpy as np


def moment_errors(U, ref, d):
    """normwise error per moment: max|U - ref| / scale, with scale = max|rho|
    for density, max(rho) * max(sound speed) for momentum, max|E| for energy"""
    rho = ref[0]
    u = ref[1:1 + d] / rho
    theta = (2.0 * ref[d + 1] - rho * (u ** 2).sum(0)) / (d * rho)
    c = np.sqrt((d + 2.0) / d * np.abs(theta))
    scales = [np.abs(rho).max()] + [np.abs(rho).max() * c.max()] * d + [np.abs(ref[d + 1]).max()]
    return np.array([np.abs(U[r] - ref[r]).max() / scales[r] for r in range(d + 2)])


def rel_inf(a, b):
    return np.abs(a - b).max() / np.abs(b).max()
