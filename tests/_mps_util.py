"""Test-side construction of isometric MPS blocks (numpy QR) and the brute-force
projection P that maps a two-site tensor to the full state vector."""
import numpy as np

import synth


def left_isometries(N_left, d, chis, seed):
    """Left-canonical A_0..A_{N_left-1}; chis[i] = right dim of site i."""
    out, cl = [], 1
    for i in range(N_left):
        cr = chis[i]
        g = synth.random_matrix(cl * d, cr, seed + i)
        q, _ = np.linalg.qr(g)
        out.append(q[:, :cr].reshape(cl, d, cr))
        cl = cr
    return out


def right_isometries(n_right, d, chis, seed):
    """Right-canonical B tensors for the last n_right sites; chis[i] = left dim of each."""
    out = []
    cr = 1
    for i in reversed(range(n_right)):
        cl = chis[i]
        g = synth.random_matrix(d * cr, cl, seed + 100 + i)
        q, _ = np.linalg.qr(g)
        out.insert(0, q[:, :cl].T.reshape(cl, d, cr))
        cr = cl
    return out


def block_left(As):
    phi = np.ones((1, 1))
    for A in As:
        cl, d, cr = A.shape
        phi = (phi @ A.reshape(cl, d * cr)).reshape(-1, cr)
    return phi  # (d^n, chi)


def block_right(Bs):
    phi = np.ones((1, 1))
    for B in reversed(Bs):
        cl, d, cr = B.shape
        phi = (B.reshape(cl * d, cr) @ phi).reshape(cl, -1)
    return phi  # (chi, d^n)
