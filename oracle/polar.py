"""Long-range (polar) part of the electron-phonon coupling, g^L (FP64).

Follows Electron Properties, the decomposition of the coupling into short- and
long-range parts and the long-range expression (after Verdi and Giustino), and
the Kokkos (Interaction) section: everything but the overlap depends on q
alone and is computed once per q; the overlap of the Bloch states is a product
of the U matrices the short-range rotation already uses.

  g^L_{nu n m}(k, q) = i L(q, nu) [U_k^dagger U_{k+q}]_{n m},

  L(q, nu) = (4 pi / V) (e^2 / 4 pi eps0) sum_s l_{s, q nu}
             sum_{G: q+G != 0} [(q+G) . Z*_s . z^s_{q nu}] e^{-(q+G).eps.(q+G) / (4 alpha)}
                                / [(q+G) . eps_inf . (q+G)],

with (q+G) in Cartesian units 2 pi (q + G)/a (a = 1 A, V = 1 A^3),
(q+G) . Z*_s . z^s = sum_{a b} (q+G)_a Z*_{s, a b} z_{s b, nu}, and l the phonon
length of the short-range coupling.

Readings taken where the paper is silent or garbled:
* the printed sum over G has no convergence factor and diverges; the Gaussian
  e^{-(q+G).eps.(q+G)/(4 alpha)} with a given alpha (A^-2), over the box of
  integer G in [-g_max, g_max]^3, is the reading;
* the printed overlap is between two states at k + q; it is read as the overlap
  of the state at k with the state at k + q, taken in the index orientation of
  the short-range coupling ([U_k^dagger U_{k+q}]_{n m}, n at k, m at k + q), so
  that g = g^S + g^L is one matrix in one orientation;
* the factor (hbar / (2 N_q m_s omega))^{1/2} is the phonon length l_{s, q nu}
  of the short-range coupling: the N_q belongs to the Bloch normalisation of
  the coarse-grid calculation, which the interpolated g^S does not carry;
* no phase of the atomic positions appears in the printed sum and none is
  used;
* modes with hbar omega < omega_min get l = 0, so L = 0 for them.
"""

import numpy as np

from .constants import E2_4PIEPS0


def g_vectors(g_max):
    """Integer reciprocal-lattice vectors of [-g_max, g_max]^3 ([n, 3] int64)."""
    ax = np.arange(-g_max, g_max + 1)
    g = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1)
    return g.reshape(-1, 3)


def polar_factor(q, z, l, born, eps_inf, alpha, g_max):
    """L(q, nu) for every q of a list.

    q [nq, 3] crystal coordinates; z [nq, 3 nat, nModes] phonon eigenvectors
    (columns); l [nq, nat, nModes] phonon lengths (0 for excluded modes);
    born [nat, 3, 3] Born effective charges (units of e); eps_inf [3, 3];
    returns [nq, nModes] complex128, in eV.
    """
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    born = np.asarray(born, dtype=np.float64)
    eps_inf = np.asarray(eps_inf, dtype=np.float64)
    nat = born.shape[0]
    G = g_vectors(g_max).astype(np.float64)
    pref = 4.0 * np.pi * E2_4PIEPS0            # (4 pi / V) e^2/(4 pi eps0), V = 1 A^3
    out = np.zeros((q.shape[0], z.shape[-1]), dtype=np.complex128)
    for i in range(q.shape[0]):
        K = 2.0 * np.pi * (q[i][None, :] + G)                  # [nG, 3] in 1/A
        keep = np.linalg.norm(K, axis=1) > 1e-12               # q + G != 0
        K = K[keep]
        den = np.einsum("ga,ab,gb->g", K, eps_inf, K)
        w = np.exp(-den / (4.0 * alpha)) / den                 # [nG]
        KZ = np.einsum("ga,sab->gsb", K, born)                 # (q+G) . Z*_s  [nG, nat, 3]
        D = np.einsum("g,gsb->sb", w, KZ).reshape(3 * nat)     # sum over G, per (s, b)
        lsa = np.repeat(l[i], 3, axis=0)                       # [3 nat, nModes]
        out[i] = pref * np.einsum("s,sv,sv->v", D, z[i], lsa)
    return out


def polar_coupling(U_k, U_kq, L):
    """g^L_{nu n m} = i L(nu) [U_k^dagger U_kq]_{n m}.

    U_k, U_kq [..., nW, nW] (eigenvectors as columns), L [..., nModes];
    returns [..., nModes, nW, nW].
    """
    O = np.conj(np.swapaxes(U_k, -1, -2)) @ U_kq               # [..., n, m]
    return 1j * L[..., :, None, None] * O[..., None, :, :]
