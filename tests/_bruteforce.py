"""Brute-force references used to pin the oracle (independent of it).

Everything here is built from first principles with numpy: the generator
matrix as an explicit Kronecker power, and maximum-likelihood decoding by
enumerating every codeword of tiny codes.
"""
import itertools

import numpy as np

F = np.array([[1, 0], [1, 1]], dtype=np.int64)


def kron_G(N: int) -> np.ndarray:
    G = np.array([[1]], dtype=np.int64)
    while G.shape[0] < N:
        G = np.kron(G, F)
    return G % 2


def encode_matrix(u: np.ndarray) -> np.ndarray:
    u = np.asarray(u, dtype=np.int64)
    return (u @ kron_G(u.shape[-1])) % 2


def codebook(frozen: np.ndarray):
    """All (u, x) pairs of the code with the given frozen mask."""
    N = len(frozen)
    free = np.where(frozen == 0)[0]
    G = kron_G(N)
    us, xs = [], []
    for bits in itertools.product([0, 1], repeat=len(free)):
        u = np.zeros(N, np.int64)
        u[free] = bits
        us.append(u)
        xs.append((u @ G) % 2)
    return np.array(us), np.array(xs)


def ml_minsum(llr: np.ndarray, frozen: np.ndarray):
    """Codeword minimising sum |llr_j| over positions where x_j disagrees with
    the hard decision (maximum likelihood on AWGN).  Returns (u, metric)."""
    us, xs = codebook(frozen)
    hd = (np.asarray(llr) < 0).astype(np.int64)
    met = (np.abs(llr)[None, :] * (xs != hd[None, :])).sum(axis=1)
    q = int(np.argmin(met))
    return us[q], float(met[q]), met


def ml_exact(llr: np.ndarray, frozen: np.ndarray):
    """Codeword maximising the likelihood: minimises sum ln(1 + e^{-(1-2x_j) llr_j})."""
    us, xs = codebook(frozen)
    s = 1 - 2 * xs
    met = np.logaddexp(0.0, -s * np.asarray(llr, np.float64)[None, :]).sum(axis=1)
    q = int(np.argmin(met))
    return us[q], float(met[q]), met
