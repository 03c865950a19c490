"""Helpers shared by the GPU tests (comparison against the FP64 oracle)."""
import math

import numpy as np

from oracle import c_oracle as C

SCHEME_ID = {"fd": C.FD, "fd2": C.FD2, "approx": C.APPROX, "interp": C.INTERP}


def oracle_gram(X, Y, scheme, order):
    """Oracle mantissa/exponent Gram of numpy paths (FP64, values as given)."""
    return C.gram(np.asarray(X, dtype=np.float64), np.asarray(Y, dtype=np.float64),
                  SCHEME_ID[scheme], order)


def rel_err_exp(m_gpu, e_gpu, m_or, e_or):
    """|m_g 2^{e_g} - m_o 2^{e_o}| / |m_o 2^{e_o}| computed without overflow."""
    m_gpu = np.asarray(m_gpu, dtype=np.float64)
    m_or = np.asarray(m_or, dtype=np.float64)
    sh = np.asarray(e_gpu, dtype=np.int64) - np.asarray(e_or, dtype=np.int64)
    g = np.ldexp(m_gpu, sh)
    return np.abs(g - m_or) / np.abs(m_or)


def rel_err(v_gpu, v_or):
    v_gpu = np.asarray(v_gpu, dtype=np.float64)
    v_or = np.asarray(v_or, dtype=np.float64)
    return np.abs(v_gpu - v_or) / np.abs(v_or)


def bm_paths(rng, n, steps, d, std):
    z = np.zeros((n, 1, d))
    return np.concatenate([z, np.cumsum(rng.normal(0.0, std, size=(n, steps, d)), axis=1)], axis=1)


def log_banner(msg):
    print(msg, flush=True)
