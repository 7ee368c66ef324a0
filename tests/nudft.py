"""Brute-force non-uniform DFT in FP64 numpy: the exact operator the NUFFT
approximates (paper Section 1: NUFFT as a fast mapping onto non-equispaced
frequencies).  Image index i_a stands for n_a = i_a - N_a/2.

    forward:  y_m = sum_n x_n exp(-i omega_m . n)
    adjoint:  x_n = sum_m y_m exp(+i omega_m . n)
"""
import numpy as np


def _phase(om, N):
    om = np.asarray(om, dtype=np.float64)
    d = len(N)
    ph = np.zeros((om.shape[0],) + tuple(N), dtype=np.float64)
    for a in range(d):
        n = np.arange(N[a], dtype=np.float64) - N[a] // 2
        shape = [1] * (d + 1)
        shape[0] = -1
        shape[a + 1] = N[a]
        ph = ph + om[:, a].reshape(-1, *([1] * d)) * n.reshape(shape)
    return ph


def nudft_forward(x, om, N, chunk=256):
    x = np.asarray(x, np.complex128).reshape(tuple(N))
    om = np.asarray(om, np.float64)
    out = np.empty(om.shape[0], np.complex128)
    for s in range(0, om.shape[0], chunk):
        ph = _phase(om[s:s + chunk], N)
        out[s:s + chunk] = (np.exp(-1j * ph) * x[None]).reshape(ph.shape[0], -1).sum(axis=1)
    return out


def nudft_adjoint(y, om, N, chunk=256):
    y = np.asarray(y, np.complex128)
    om = np.asarray(om, np.float64)
    out = np.zeros(tuple(N), np.complex128)
    for s in range(0, om.shape[0], chunk):
        ph = _phase(om[s:s + chunk], N)
        out += (np.exp(1j * ph) * y[s:s + chunk].reshape(-1, *([1] * len(N)))).sum(axis=0)
    return out


def rel_l2(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
