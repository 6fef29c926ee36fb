"""Seeded tensor-variate inputs of the eigenvalue solve: the per-axis Gram
spectra E_l (the squared singular values of each axis' unfolding, Algorithm 1's
first loop) of synthetic tensors.

* low_rank_tensor_spectra: a sum of `rank` rank-one tensors with weights
  2^-q plus Gaussian noise; every axis' spectrum has the same trace |X|^2, so
  a single modality over all axes is balanced (every shift direction is flat).
* coil_like_spectra: the shape of the paper's COIL-20 experiment, 20 objects
  of 72 frames x 128 x 128 pixels as modalities (frame, row_i, col_i) sharing
  the frame axis (41 axes).  Each object is a rotation: every pixel varies with
  the frame angle through the first three circular harmonics, with a rank-3
  image per harmonic and Gaussian noise.  It stands in for the image data,
  which is not used.
"""
import numpy as np


def _spectrum(U):
    e = np.linalg.eigvalsh(U @ U.T)[::-1]
    return np.ascontiguousarray(np.maximum(e, 0.0))


def low_rank_tensor_spectra(shape, rank, seed, noise=0.3):
    rng = np.random.default_rng(seed)
    fac = [rng.standard_normal((d, rank)) for d in shape]
    X = np.zeros(shape)
    for q in range(rank):
        t = fac[0][:, q]
        for f in fac[1:]:
            t = np.multiply.outer(t, f[:, q])
        X += t * 2.0 ** -q
    X += noise * rng.standard_normal(shape)
    return [_spectrum(np.moveaxis(X, l, 0).reshape(shape[l], -1)) for l in range(len(shape))]


def coil_like_spectra(n_obj=20, frames=72, h=128, w=128, seed=0, noise=0.05):
    """Returns (E, modalities): E[0] the frame axis, E[1 + 2i] and E[2 + 2i]
    object i's row and column axes; modality i = (0, 1 + 2i, 2 + 2i).  The
    tensors come from synth.rotating_objects."""
    import synth
    G_frame = np.zeros((frames, frames))
    rows, cols = [], []
    for X in synth.rotating_objects(n_obj, frames, h, w, seed=seed, noise=noise):
        U = X.reshape(frames, -1)
        G_frame += U @ U.T
        rows.append(_spectrum(np.moveaxis(X, 1, 0).reshape(h, -1)))
        cols.append(_spectrum(np.moveaxis(X, 2, 0).reshape(w, -1)))
    E = [np.ascontiguousarray(np.maximum(np.linalg.eigvalsh(G_frame)[::-1], 0.0))]
    mods = []
    for i in range(n_obj):
        E += [rows[i], cols[i]]
        mods.append((0, 1 + 2 * i, 2 + 2 * i))
    return E, mods
