"""Seeded synthetic systems shaped like the paper's el-ph workloads.

Conventions (shared by every consumer of these arrays):

* simple-cubic Bravais lattice, a = 1 Angstrom; lattice vectors R, wavevectors
  k, q and atomic positions are in crystal (= Cartesian, since a = 1) units;
* lattice-vector lists are int32 [n, 3], ordered with the last component
  fastest, so ``box_vectors(r)`` enumerates [-r, r]^3;
* H(R): complex128 [n_rh, nW, nW] in eV with H(-R) = H(R)^dagger;
* Phi(R): float64 [n_rd, 3 nat, 3 nat] in eV/A^2, phonon index s*3 + alpha
  (atom-major), Phi(0|s'R)_{s s'} = Phi(-R)_{s' s}^T and the acoustic sum rule
  sum_{R s'} Phi(R)_{s s'} = 0 built in;
* masses: float64 [nat] in amu;
* g(Re, Rp): complex128 [n_re, n_rp, 3 nat, nW, nW] in eV/A; the first Wannier
  index pairs with k, the second with k+q.

Random tensors use CN(0,1) = (N(0,1) + i N(0,1)) / sqrt(2) scaled by an
exponential decay in the Cartesian length |R|.  Every draw comes from a numpy
PCG64 stream keyed by (seed, tensor tag, block index), so results do not depend
on the number of threads used to fill large tensors.

Force constants come from a Born-von Karman model: every bond b between atoms
at distance in a chosen shell gets a spring constant k_b ~ U[0.5, 1.5] eV/A^2
and a bond tensor K_b = k_b [r r^T + 0.25 (1 - r r^T)] (r the unit bond
vector).  The transverse quarter keeps nearest-neighbour-only lattices free of
spurious zero modes; any positive-definite bond tensor gives a positive
semi-definite dynamical matrix.
"""

from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

# tags that separate the random streams of one system
_TAG_MASS, _TAG_SPRING, _TAG_H, _TAG_G, _TAG_POS, _TAG_POLAR = 11, 12, 13, 14, 15, 16


def _rng(seed: int, tag: int, block: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, tag, block])))


def box_vectors(r: int) -> np.ndarray:
    """All integer vectors of [-r, r]^3, last component fastest (int32 [(2r+1)^3, 3])."""
    ax = np.arange(-r, r + 1, dtype=np.int32)
    g = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1)
    return np.ascontiguousarray(g.reshape(-1, 3))


@dataclass
class System:
    """One synthetic crystal: everything the el-ph path reads (host numpy arrays)."""

    n_wannier: int
    n_atoms: int
    positions: np.ndarray            # [nat, 3] crystal coordinates
    mass: np.ndarray                 # [nat] amu
    rh: np.ndarray                   # [n_rh, 3] int32
    h_r: np.ndarray                  # [n_rh, nW, nW] complex128, eV
    rd: np.ndarray                   # [n_rd, 3] int32
    phi_r: np.ndarray                # [n_rd, 3nat, 3nat] float64, eV/A^2
    re: np.ndarray                   # [n_re, 3] int32
    rp: np.ndarray                   # [n_rp, 3] int32
    g_rr: np.ndarray                 # [n_re, n_rp, 3nat, nW, nW] complex128, eV/A
    meta: dict = field(default_factory=dict)
    # polar crystals only (None otherwise): Born effective charges [nat, 3, 3] (e),
    # high-frequency dielectric tensor [3, 3], the Gaussian damping parameter of
    # the sum over G (A^-2) and the half-width of the integer G box
    born: np.ndarray = None
    eps_inf: np.ndarray = None
    ewald_alpha: float = 0.0
    g_max: int = 0

    @property
    def n_modes(self) -> int:
        return 3 * self.n_atoms


# ----------------------------------------------------------------------------
# structures
# ----------------------------------------------------------------------------

def cscl_structure():
    """Two atoms, CsCl arrangement; nearest-neighbour shell sqrt(3)/2."""
    pos = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])
    return pos, [math.sqrt(3.0) / 2.0]


def perovskite_structure():
    """Cubic perovskite ABO3 (5 atoms); shells 0.5 (B-O) and sqrt(2)/2 (A-O, O-O)."""
    pos = np.array([
        [0.0, 0.0, 0.0],
        [0.5, 0.5, 0.5],
        [0.5, 0.5, 0.0],
        [0.5, 0.0, 0.5],
        [0.0, 0.5, 0.5],
    ])
    return pos, [0.5, math.sqrt(2.0) / 2.0]


def random_structure(seed: int, n_atoms: int, min_sep: float = 0.25, cutoff: float = 1.01):
    """n_atoms random positions in the unit cell, pairwise periodic distance >= min_sep.

    Bonds are drawn to every neighbour closer than ``cutoff`` (returned as a
    single open shell ``('cutoff', cutoff)``).  The default 1.01 A includes each
    atom's own periodic images along the axes, which keeps the spring network
    free of soft modes away from q = 0.
    """
    rng = _rng(seed, _TAG_POS)
    for _ in range(10000):
        pos = rng.uniform(0.0, 1.0, size=(n_atoms, 3))
        ok = True
        for a in range(n_atoms):
            for b in range(a + 1, n_atoms):
                d = pos[b] - pos[a]
                d -= np.round(d)
                if np.linalg.norm(d) < min_sep:
                    ok = False
        if ok:
            return pos, ("cutoff", cutoff)
    raise RuntimeError("could not place atoms")


def _bonds(pos: np.ndarray, shells, rmax: int = 1):
    """Unique bonds (s, s', R, d) with d = pos[s'] + R - pos[s] in a shell.

    A bond and its reverse (s', s, -R) are one bond; the representative is the
    lexicographically smaller tuple.
    """
    nat = pos.shape[0]
    out = []
    tol = 1e-9
    for s in range(nat):
        for s2 in range(nat):
            for R in box_vectors(rmax):
                if s == s2 and not R.any():
                    continue
                d = pos[s2] + R - pos[s]
                dist = float(np.linalg.norm(d))
                if isinstance(shells, tuple) and shells and shells[0] == "cutoff":
                    hit = dist < shells[1]
                else:
                    hit = any(abs(dist - sh) < tol for sh in shells)
                if not hit:
                    continue
                key = (s, s2, tuple(int(x) for x in R))
                rkey = (s2, s, tuple(int(-x) for x in R))
                if key < rkey:
                    out.append((s, s2, np.array(R, dtype=np.int32), d))
    return out


def born_von_karman(seed: int, pos: np.ndarray, shells, rmax: int = 1,
                    transverse: float = 0.25, spring_range=(0.5, 1.5)):
    """Force constants Phi(R) of a bond-spring model with the acoustic sum rule.

    Returns (rd [n_rd,3] int32, phi_r [n_rd,3nat,3nat]).  rd is box_vectors(rmax).
    """
    nat = pos.shape[0]
    rd = box_vectors(rmax)
    index = {tuple(int(x) for x in r): i for i, r in enumerate(rd)}
    phi = np.zeros((rd.shape[0], 3 * nat, 3 * nat))
    rng = _rng(seed, _TAG_SPRING)
    bonds = _bonds(pos, shells, rmax)
    if not bonds:
        raise ValueError("no bonds in the requested shells")
    i0 = index[(0, 0, 0)]
    for (s, s2, R, d) in bonds:
        kb = rng.uniform(*spring_range)
        rhat = d / np.linalg.norm(d)
        P = np.outer(rhat, rhat)
        K = kb * (P + transverse * (np.eye(3) - P))
        iR = index[tuple(int(x) for x in R)]
        imR = index[tuple(int(-x) for x in R)]
        phi[iR, 3 * s:3 * s + 3, 3 * s2:3 * s2 + 3] -= K
        phi[imR, 3 * s2:3 * s2 + 3, 3 * s:3 * s + 3] -= K
        phi[i0, 3 * s:3 * s + 3, 3 * s:3 * s + 3] += K
        phi[i0, 3 * s2:3 * s2 + 3, 3 * s2:3 * s2 + 3] += K
    return rd, phi


# ----------------------------------------------------------------------------
# random tensors
# ----------------------------------------------------------------------------

def _cn(rng: np.random.Generator, shape) -> np.ndarray:
    x = rng.standard_normal(size=tuple(shape) + (2,))
    return (x[..., 0] + 1j * x[..., 1]) / math.sqrt(2.0)


def hamiltonian_r(seed: int, rvecs: np.ndarray, n_wannier: int, decay: float) -> np.ndarray:
    """H(R) = CN entries x exp(-|R|/decay), with H(-R) = H(R)^dagger, H(0) Hermitian.

    ``rvecs`` must be closed under R -> -R.  The first of each +-R pair (in list
    order) carries the draw.
    """
    index = {tuple(int(x) for x in r): i for i, r in enumerate(rvecs)}
    h = np.zeros((rvecs.shape[0], n_wannier, n_wannier), dtype=np.complex128)
    done = np.zeros(rvecs.shape[0], dtype=bool)
    rng = _rng(seed, _TAG_H)
    for i, r in enumerate(rvecs):
        if done[i]:
            continue
        j = index.get(tuple(int(-x) for x in r))
        if j is None:
            raise ValueError("R set is not closed under inversion")
        B = _cn(rng, (n_wannier, n_wannier)) * math.exp(-float(np.linalg.norm(r)) / decay)
        if i == j:
            h[i] = 0.5 * (B + B.conj().T)
        else:
            h[i] = B
            h[j] = B.conj().T
        done[i] = done[j] = True
    return h


def coupling_r(seed: int, re: np.ndarray, rp: np.ndarray, n_modes: int, n_wannier: int,
               decay_e: float, decay_p: float, threads: int = 8) -> np.ndarray:
    """g(Re, Rp) = CN entries x exp(-|Re|/decay_e - |Rp|/decay_p), no symmetry imposed.

    Block ire is drawn from its own stream (seed, tag, ire), so the tensor is the
    same for any thread count.
    """
    n_re, n_rp = re.shape[0], rp.shape[0]
    out = np.empty((n_re, n_rp, n_modes, n_wannier, n_wannier), dtype=np.complex128)
    le = np.linalg.norm(re.astype(np.float64), axis=1)
    lp = np.linalg.norm(rp.astype(np.float64), axis=1)
    dp = np.exp(-lp / decay_p)

    def fill(ire: int) -> None:
        rng = _rng(seed, _TAG_G, ire)
        x = rng.standard_normal(size=(n_rp, n_modes, n_wannier, n_wannier, 2))
        scale = (math.exp(-le[ire] / decay_e) / math.sqrt(2.0)) * dp
        blk = out[ire]
        blk.real[...] = x[..., 0] * scale[:, None, None, None]
        blk.imag[...] = x[..., 1] * scale[:, None, None, None]

    if threads <= 1 or n_re < 4:
        for i in range(n_re):
            fill(i)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(fill, range(n_re)))
    return out


# ----------------------------------------------------------------------------
# systems
# ----------------------------------------------------------------------------

def make_system(seed: int, n_wannier: int, positions: np.ndarray, shells, r_h: int, r_e: int,
                r_p: int, decay_h: float = 1.0, decay_g: float = 0.8,
                mass_range=(1.0, 3.0), threads: int = 8, with_coupling: bool = True) -> System:
    nat = positions.shape[0]
    mass = _rng(seed, _TAG_MASS).uniform(*mass_range, size=nat)
    rd, phi = born_von_karman(seed, positions, shells)
    rh = box_vectors(r_h)
    h_r = hamiltonian_r(seed, rh, n_wannier, decay_h)
    re = box_vectors(r_e)
    rp = box_vectors(r_p)
    g = (coupling_r(seed, re, rp, 3 * nat, n_wannier, decay_g, decay_g, threads=threads)
         if with_coupling else None)
    return System(n_wannier=n_wannier, n_atoms=nat, positions=positions, mass=mass,
                  rh=rh, h_r=h_r, rd=rd, phi_r=phi, re=re, rp=rp, g_rr=g,
                  meta=dict(seed=seed, r_h=r_h, r_e=r_e, r_p=r_p))


def config_c1(seed: int = 1) -> System:
    """Toy model: CsCl (2 atoms, 6 modes), nW = 4, R in [-1,1]^3 (27) for H and g."""
    pos, shells = cscl_structure()
    return make_system(seed, 4, pos, shells, r_h=1, r_e=1, r_p=1)


def config_c2(seed: int = 2, threads: int = 8, with_coupling: bool = True) -> System:
    """Realistic size: perovskite (5 atoms, 15 modes), nW = 16, R in [-3,3]^3 (343).

    g(Re, Rp) is [343, 343, 15, 16, 16] complex128 (7.23 GB).
    """
    pos, shells = perovskite_structure()
    return make_system(seed, 16, pos, shells, r_h=3, r_e=3, r_p=3, threads=threads,
                       with_coupling=with_coupling)


def small_system(seed: int, n_wannier: int = 3, n_atoms: int = 2, r: int = 1) -> System:
    """Small random system for parity/property tests (nat 1, 2 or 5 use fixed structures)."""
    if n_atoms == 2:
        pos, shells = cscl_structure()
    elif n_atoms == 5:
        pos, shells = perovskite_structure()
    elif n_atoms == 1:
        pos, shells = np.zeros((1, 3)), [1.0]
    else:
        pos, shells = random_structure(seed, n_atoms)
    return make_system(seed, n_wannier, pos, shells, r_h=r, r_e=r, r_p=r)


def local_coupling_system(seed: int, n_wannier: int = 3, onsite_gap: float = 1.5,
                          hop_scale: float = 0.1) -> System:
    """CsCl system whose |g|^2 varies smoothly over the q mesh.

    The random system of ``small_system`` with its hoppings scaled by ``hop_scale``
    and on-site levels 0, gap, 2 gap, ... added at R = 0 (bands well separated,
    eigenvectors close to the Wannier basis), and g(Re, Rp) kept at Re = 0 only
    (coupling local in the electron index).  Used where a learnable coupling
    structure is needed.
    """
    s = small_system(seed, n_wannier=n_wannier, n_atoms=2, r=1)
    z = int(np.nonzero((s.rh == 0).all(axis=1))[0][0])
    s.h_r = s.h_r * hop_scale
    s.h_r[z] += np.diag(onsite_gap * np.arange(n_wannier, dtype=np.float64))
    ze = int(np.nonzero((s.re == 0).all(axis=1))[0][0])
    s.re = np.ascontiguousarray(s.re[ze:ze + 1])
    s.g_rr = np.ascontiguousarray(s.g_rr[ze:ze + 1])
    s.meta.update(kind="local-coupling", onsite_gap=onsite_gap, hop_scale=hop_scale)
    return s


def config_c4_specs(base_seed: int = 400, count: int = 32, per_system_cap: float = 1.5e9,
                    total_cap: float = 24e9):
    """Sizes of the batched workload's independent systems (arrays built by ``config_c4``).

    nW ~ U{4..24}, nat ~ U{2..10} (nModes 6..30), H(R) box r_h ~ U{2,3,4}
    (125..729 vectors), g(Re,Rp) box r_g ~ U{2,3,4}, mesh ~ U{16..32}^3.  A
    system whose complex128 g(Re,Rp) exceeds ``per_system_cap`` bytes redraws
    (nW, nat, r_g) from its own stream until it fits; the total is then capped at
    ``total_cap`` by shrinking the largest systems the same way.  (Uncapped, the
    largest draws need ~150 GB each: more than one GPU holds.)
    """
    specs = []

    def nbytes(sp):
        nr = (2 * sp["r_g"] + 1) ** 3
        return nr * nr * 3 * sp["n_atoms"] * sp["n_wannier"] ** 2 * 16

    for i in range(count):
        rng = _rng(base_seed + i, 99)
        sp = dict(seed=base_seed + i, n_wannier=int(rng.integers(4, 25)),
                  n_atoms=int(rng.integers(2, 11)), r_h=int(rng.integers(2, 5)),
                  r_g=int(rng.integers(2, 5)), mesh=int(rng.integers(16, 33)))
        while nbytes(sp) > per_system_cap:
            sp["n_wannier"] = int(rng.integers(4, 25))
            sp["n_atoms"] = int(rng.integers(2, 11))
            sp["r_g"] = int(rng.integers(2, 5))
        specs.append(sp)
    while sum(nbytes(sp) for sp in specs) > total_cap:
        j = max(range(count), key=lambda k: nbytes(specs[k]))
        rng = _rng(specs[j]["seed"], 98)
        specs[j]["r_g"] = max(2, specs[j]["r_g"] - 1)
        if nbytes(specs[j]) > per_system_cap / 4:
            specs[j]["n_wannier"] = max(4, specs[j]["n_wannier"] // 2)
    return specs


def config_c4(spec: dict, threads: int = 8) -> System:
    """One system of the batched workload from its spec (random positions, bonds < 1.01 A)."""
    pos, shells = random_structure(spec["seed"], spec["n_atoms"])
    s = make_system(spec["seed"], spec["n_wannier"], pos, shells, r_h=spec["r_h"],
                    r_e=spec["r_g"], r_p=spec["r_g"], threads=threads)
    s.meta["mesh"] = (spec["mesh"],) * 3
    return s


def add_polar(system: System, seed: int, alpha: float = 5.0, g_max: int = 3,
              eps_scale: float = 4.0) -> System:
    """Give a system Born effective charges and a dielectric tensor (in place).

    Z*_s = diag(d_s) + 0.3 N(0,1)^{3x3} with d_s ~ U[1, 3] and alternating
    signs, then the mean over atoms removed (charge neutrality, sum_s Z*_s = 0);
    eps_inf = eps_scale I + A A^T / 6 with A ~ N(0,1)^{3x3} (symmetric positive
    definite).  alpha and g_max set the damping and the box of the G sum.
    """
    rng = _rng(seed, _TAG_POLAR)
    nat = system.n_atoms
    d = rng.uniform(1.0, 3.0, size=nat) * np.where(np.arange(nat) % 2 == 0, 1.0, -1.0)
    Z = np.stack([np.diag(np.full(3, d[s_])) for s_ in range(nat)]) + \
        0.3 * rng.standard_normal((nat, 3, 3))
    Z -= Z.mean(axis=0, keepdims=True)
    A = rng.standard_normal((3, 3))
    system.born = np.ascontiguousarray(Z)
    system.eps_inf = eps_scale * np.eye(3) + A @ A.T / 6.0
    system.ewald_alpha = float(alpha)
    system.g_max = int(g_max)
    system.meta.update(polar=True)
    return system


_TAG_PHI3 = 17


def third_order_constants(seed: int, n_atoms: int, r_src: int = 1, decay: float = 0.8):
    """Phi3(s a R, s' b R', s'' c 0) symmetric under every permutation of its three displacements.

    A random A0(x1, R1 - R3, x2, R2 - R3, x3) ~ N(0,1) exp(-(|R1-R3| + |R2-R3|)/decay)
    is drawn for relative vectors in [-r_src, r_src]^3 and averaged over the six
    orderings of the three (index, cell) pairs, each translated so that its third
    cell is the reference cell; the result is stored for R, R' in
    [-2 r_src, 2 r_src]^3, which holds every non-zero entry.
    Returns (r [n, 3] int32, phi3 [n, n, 3nat, 3nat, 3nat] float64 eV/A^3).
    """
    nm = 3 * n_atoms
    src = box_vectors(r_src)
    ns = src.shape[0]
    rng = _rng(seed, _TAG_PHI3)
    dec = np.exp(-np.linalg.norm(src.astype(np.float64), axis=1) / decay)
    A0 = rng.standard_normal((ns, ns, nm, nm, nm)) * (dec[:, None] * dec[None, :])[:, :, None, None, None]
    sidx = {tuple(int(x) for x in v): i for i, v in enumerate(src)}
    r = box_vectors(2 * r_src)
    n = r.shape[0]
    phi = np.zeros((n, n, nm, nm, nm))

    def a0(d1, d2):
        i, j = sidx.get(tuple(int(x) for x in d1)), sidx.get(tuple(int(x) for x in d2))
        return None if i is None or j is None else A0[i, j]

    z = np.zeros(3, dtype=np.int64)
    for i, R in enumerate(r):
        for j, Rp in enumerate(r):
            acc = np.zeros((nm, nm, nm))
            # orderings of (x1, R) (x2, R') (x3, 0); each term is A0 of the ordering
            # with its third cell moved to the reference cell, axes back in (x1, x2, x3) order
            for (c1, c2, c3), perm in (((R, Rp, z), (0, 1, 2)), ((Rp, R, z), (1, 0, 2)),
                                       ((R, z, Rp), (0, 2, 1)), ((z, R, Rp), (2, 0, 1)),
                                       ((Rp, z, R), (1, 2, 0)), ((z, Rp, R), (2, 1, 0))):
                blk = a0(c1 - c3, c2 - c3)
                if blk is not None:
                    acc += np.transpose(blk, np.argsort(perm))
            phi[i, j] = acc / 6.0
    return r, phi
