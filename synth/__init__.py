"""Seeded synthetic inputs shared by the GPU path's tests/bench and the CPU oracle.

This module holds random-number generation and the construction of the synthetic
workloads only. It contains none of the method's arithmetic (no contraction, SVD,
entropy, controller or sweep): it produces the bytes that both sides receive.

Generator: splitmix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) used counter-style, value_i = mix(seed + (i+1)*golden),
mapped to 53-bit uniforms in (0, 1] and to normals by the Box-Muller transform
(Box & Muller 1958), both outputs of each pair used in order.
"""
from __future__ import annotations

import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Counter-based splitmix64 outputs for counters start+1 .. start+count."""
    with np.errstate(over="ignore"):
        ctr = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + ctr * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform53(seed: int, start: int, count: int) -> np.ndarray:
    """Uniforms in (0, 1] with 53 random bits: ((x >> 11) + 1) * 2^-53."""
    x = splitmix64(seed, start, count)
    return ((x >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)


def normal(seed: int, count: int, start: int = 0) -> np.ndarray:
    """`count` standard normals from stream `seed`, Box-Muller on consecutive uniform pairs."""
    npair = (count + 1) // 2
    u = uniform53(seed, 2 * start, 2 * npair)
    u1, u2 = u[0::2], u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * npair)
    z[0::2] = r * np.cos(2.0 * math.pi * u2)
    z[1::2] = r * np.sin(2.0 * math.pi * u2)
    return z[:count]


# ----------------------------------------------------------------------------
# Random initial MPS (open chain): A_i has shape (chi_{i-1}, d, chi_i),
# chi_b = min(chi_init, d^(b+1), d^(N-1-b)), entries iid N(0,1) consumed in
# site-major, row-major order from one stream.
# ----------------------------------------------------------------------------
def initial_bond_dims(N: int, d: int, chi_init: int) -> list[int]:
    return [min(chi_init, d ** (b + 1), d ** (N - 1 - b)) for b in range(N - 1)]


def random_mps(N: int, d: int, chi_init: int, seed: int = 0):
    """Returns (packed float64 array, bond dims list, per-site shapes)."""
    chi = initial_bond_dims(N, d, chi_init)
    shapes = []
    for i in range(N):
        cl = 1 if i == 0 else chi[i - 1]
        cr = 1 if i == N - 1 else chi[i]
        shapes.append((cl, d, cr))
    total = sum(a * b * c for a, b, c in shapes)
    return normal(seed, total), chi, shapes


# ----------------------------------------------------------------------------
# Isolated-SVD test matrices: A = U diag(sigma) V^T, sigma_k = exp(-k/tau),
# U and V Haar-distributed orthogonal matrices obtained as Householder products
# (QR of a Gaussian matrix from the stream, columns sign-fixed by diag(R)).
# ----------------------------------------------------------------------------
def _householder_orthogonal(n: int, seed: int, stream: int) -> np.ndarray:
    g = normal(seed * 1000003 + stream, n * n).reshape(n, n)
    q, r = np.linalg.qr(g)
    q *= np.sign(np.diag(r))[None, :]
    return q


def svd_test_spectrum(n: int, tau: float) -> np.ndarray:
    return np.exp(-np.arange(n, dtype=np.float64) / tau)


def svd_test_matrix(n: int, tau: float, seed: int = 0, index: int = 0) -> np.ndarray:
    """FP64 n x n matrix with prescribed spectrum exp(-k/tau). `index` selects the
    batch member: U from stream 2*index, V from stream 2*index+1."""
    u = _householder_orthogonal(n, seed, 2 * index)
    v = _householder_orthogonal(n, seed, 2 * index + 1)
    s = svd_test_spectrum(n, tau)
    return (u * s[None, :]) @ v.T


def random_matrix(m: int, n: int, seed: int) -> np.ndarray:
    return normal(seed, m * n).reshape(m, n)


# ----------------------------------------------------------------------------
# Batched-chain workload: XXZ chains with anisotropy uniform in [0, 2] and
# length uniform over {32, 48, 64, 96, 128}, both drawn from stream `seed`.
# ----------------------------------------------------------------------------
CHAIN_LENGTHS = (32, 48, 64, 96, 128)


def xxz_chain_set(n_chains: int = 64, seed: int = 0, lengths=CHAIN_LENGTHS):
    u = uniform53(seed, 0, 2 * n_chains)
    out = []
    for c in range(n_chains):
        delta = 2.0 * u[2 * c]
        idx = min(int(u[2 * c + 1] * len(lengths)), len(lengths) - 1)
        out.append((float(delta), int(lengths[idx])))
    return out


# ----------------------------------------------------------------------------
# Circuit workload: a hardware-efficient ansatz of real gates (single-qubit
# rotations RY(theta) = [[cos theta/2, -sin theta/2], [sin theta/2, cos theta/2]]
# and CNOTs, control on the left qubit), as a list of ops.  One ansatz layer is
# two ops: parity 0 applies CNOT (RY x RY) to the pairs (0,1), (2,3), ...;
# parity 1 applies CNOT to (1,2), (3,4), ... (and, for odd N, the last qubit's
# rotation before its CNOT).  Angles uniform in [0, 2 pi) from stream `seed`,
# one per qubit per layer.  Gates are real 4 x 4 matrices G[2s+t][2s'+t'],
# packed op after op in increasing bond.
# ----------------------------------------------------------------------------
_CNOT = np.array([[1.0, 0, 0, 0], [0, 1.0, 0, 0], [0, 0, 0, 1.0], [0, 0, 1.0, 0]])


def ry(theta: float) -> np.ndarray:
    c, s = math.cos(0.5 * theta), math.sin(0.5 * theta)
    return np.array([[c, -s], [s, c]])


def hea_circuit(N: int, layers: int, seed: int = 0):
    """Returns (parity list, packed gates (float64), angles (layers x N))."""
    ang = 2.0 * math.pi * uniform53(seed, 0, layers * N).reshape(layers, N)
    parity, gates = [], []
    eye = np.eye(2)
    for l in range(layers):
        parity.append(0)
        for b in range(0, N - 1, 2):
            gates.append(_CNOT @ np.kron(ry(ang[l, b]), ry(ang[l, b + 1])))
        parity.append(1)
        for b in range(1, N - 1, 2):
            left = eye
            right = ry(ang[l, b + 1]) if (N % 2 == 1 and b + 1 == N - 1) else eye
            gates.append(_CNOT @ np.kron(left, right))
    g = np.concatenate([x.ravel() for x in gates]) if gates else np.zeros(0)
    return parity, g, ang
