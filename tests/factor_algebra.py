"""Dense-matrix forms of the paper's factorisation building blocks (numpy).

These restate Eq. 2 and the Stockham stage in matrix form so the index
conventions used by the GPU kernels can be checked on the CPU at tiny N.
"""
import numpy as np


def dft_matrix(n, sign=-1):
    """Section II definition: entry (m, k) = w_N^{m k}, w_N = exp(sign 2 pi i/N)."""
    m = np.arange(n)
    e = np.outer(m, m) % n
    return np.exp(sign * 2j * np.pi * e / n)


def stride_perm(n, k):
    """Pi^N_K: (Pi x)[i M + j] = x[j K + i], i < K, j < M (gather at stride K)."""
    m = n // k
    p = np.zeros((n, n))
    for i in range(k):
        for j in range(m):
            p[i * m + j, j * k + i] = 1
    return p


def twiddle_diag(n, m, sign=-1):
    """D^N_M: diag(w_N^{i j}) at position i M + j, i < N/M, j < M."""
    k = n // m
    d = np.array([np.exp(sign * 2j * np.pi * ((i * j) % n) / n) for i in range(k) for j in range(m)])
    return np.diag(d)


def eq2(n, k, sign=-1):
    """(DFT_K (x) I_M) D^N_M (I_K (x) DFT_M) Pi^N_K with N = M K."""
    m = n // k
    return (np.kron(dft_matrix(k, sign), np.eye(m)) @ twiddle_diag(n, m, sign)
            @ np.kron(np.eye(k), dft_matrix(m, sign)) @ stride_perm(n, k))


def stockham_stage_matrix(n, r, ns, sign=-1):
    """Stage with radix r after ns = product of the earlier radices.

    Index form: for j < N/R, k = j mod Ns,
        v_s = x[j + s N/R] * w_{Ns R}^{s k},  v <- DFT_R v,
        y[(j div Ns) Ns R + s Ns + k] = v_s.
    """
    s_mat = np.zeros((n, n), np.complex128)
    nr = n // r
    w = dft_matrix(r, sign)
    for j in range(nr):
        k = j % ns
        base = (j // ns) * ns * r + k
        for s_out in range(r):
            for s_in in range(r):
                tw = np.exp(sign * 2j * np.pi * ((s_in * k) % (ns * r)) / (ns * r))
                s_mat[base + s_out * ns, j + s_in * nr] += w[s_out, s_in] * tw
    return s_mat


def stockham_stage_kron(n, r, ns, sign=-1):
    """Same stage in Kronecker form: (L^{mR}_m (x) I_Ns)(DFT_R (x) I_{N/R}) T,
    m = N/(R Ns), L^{ab}_a the stride permutation (L x)[i b + j] = x[j a + i]."""
    m = n // (r * ns)
    # T: element j + s N/R scaled by w_{Ns R}^{s (j mod Ns)}
    nr = n // r
    t = np.array([np.exp(sign * 2j * np.pi * ((s * (j % ns)) % (ns * r)) / (ns * r))
                  for s in range(r) for j in range(nr)])
    l_perm = stride_perm(m * r, m)     # L^{mR}_m gathers at stride m
    return np.kron(l_perm, np.eye(ns)) @ np.kron(dft_matrix(r, sign), np.eye(nr)) @ np.diag(t)


def stockham_product(n, radices, sign=-1):
    p = np.eye(n, dtype=np.complex128)
    ns = 1
    for r in radices:
        p = stockham_stage_matrix(n, r, ns, sign) @ p
        ns *= r
    assert ns == n
    return p
