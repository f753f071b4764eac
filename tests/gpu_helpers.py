"""Shared helpers of the GPU parity tests (marshalling and norms only)."""
import numpy as np

from paper_2306_01959_amd import scene


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def fmix32(v):
    """MurmurHash3 32-bit finaliser (numpy, uint32 arithmetic)."""
    v = np.asarray(v, np.uint64) & 0xFFFFFFFF
    v ^= v >> 16
    v = (v * 0x85EBCA6B) & 0xFFFFFFFF
    v ^= v >> 13
    v = (v * 0xC2B2AE35) & 0xFFFFFFFF
    v ^= v >> 16
    return v.astype(np.uint32)


def set_stats(pairs, n, is_bnd):
    """Per-particle (fluid count, boundary count, id hash) of an (i, j) pair
    set, with the interaction's pair rule: boundary i keeps fluid j only."""
    nf = np.zeros(n, np.int64)
    nb = np.zeros(n, np.int64)
    hs = np.zeros(n, np.uint64)
    if pairs:
        ij = np.array(sorted(pairs), dtype=np.int64)
        i, j = ij[:, 0], ij[:, 1]
        keep = ~(is_bnd[i] & is_bnd[j])
        i, j = i[keep], j[keep]
        np.add.at(nf, i[~is_bnd[j]], 1)
        np.add.at(nb, i[is_bnd[j]], 1)
        np.add.at(hs, i, fmix32(j).astype(np.uint64))
    return nf, nb, (hs & 0xFFFFFFFF).astype(np.uint32)


def scene_from_oracle(st, params, name="developed"):
    """Scene holding an oracle state's current level (original order) and a
    dict with its previous level."""
    sc = scene.Scene(name, st.x.copy(), st.y.copy(), st.z.copy(), st.ux.copy(), st.uy.copy(),
                     st.uz.copy(), st.rho.copy(), st.is_bnd.astype(bool), dict(params))
    prev = dict(ux=st.uxm.copy(), uy=st.uym.copy(), uz=st.uzm.copy(), rho=st.rhom.copy())
    return sc, prev
