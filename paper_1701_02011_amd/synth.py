"""Seeded synthetic inputs for the DSRG-MRPT3 hot path.

This module only *draws* inputs; it holds none of the method's arithmetic.
It is shared by the FP64 oracle, the tests and the benchmark, so that both
sides of every parity check see bit-identical inputs.

What is drawn (all FP64, spatial orbitals ordered [core | active | virtual]):

* ``eps``   -- semicanonical orbital energies, one sorted uniform draw per block
  (the zeroth-order Hamiltonian is the diagonal of the Fock operator in each
  block, Sec. II.B, Eq. F0th).
* ``B``     -- the three-index factorised integrals B^Q_pq, symmetric in pq,
  i.i.d. N(0, 0.1^2) on the upper triangle, so (pq|rs) = sum_Q B^Q_pq B^Q_rs
  (Sec. III, Eq. int_fact).
* ``ci``    -- a random normalised CAS(n,n) vector over all determinants with
  n_alpha = ceil(n/2), n_beta = floor(n/2) electrons in the n active orbitals
  (Sec. II.A, Eq. mref).  The reference is core^2 x CAS x virtual^0.
* ``gamma1``, ``gamma2``, ``gamma3`` -- the active-space 1-, 2- and 3-body
  reduced density matrices of that vector in the spin-block layout the library
  takes as input (see include/dsrg.h).  The paper poses the reference only
  through its densities (Sec. I: any reference whose one-, two- and three-body
  cumulants are available can be used); building them from a CI vector is part
  of making the input, not of the method.

Fock-space conventions used for the RDMs: the 2*nA active spin orbitals are
bits 0..nA-1 (alpha) and nA..2nA-1 (beta); a creation operator on bit k picks up
the sign (-1)^(number of occupied bits below k).  A determinant with the
alpha string S_a and beta string S_b is the product of creators in ascending bit
order acting on the vacuum.

Spin-block layout of the densities (spatial indices u,v,w,x,y,z in [0,nA)):

* gamma1[s][u][v]            = <a+_{u s} a_{v s}>,                 s in (alpha, beta)
* gamma2[b][u][v][x][y]      = <a+_{u s1} a+_{v s2} a_{y s2} a_{x s1}>, b in (aa, ab, bb)
* gamma3[b][u][v][w][x][y][z]= <a+_{u s1} a+_{v s2} a+_{w s3} a_{z s3} a_{y s2} a_{x s1}>,
                               b in (aaa, aab, abb, bbb)
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Problem",
    "CONFIGS",
    "make_problem",
    "make_config",
    "make_batch_config",
    "batch_sizes",
    "random_ci",
    "active_rdms",
    "fock_rdms",
    "det_strings",
]


@dataclasses.dataclass
class Problem:
    """One DSRG-MRPT3 problem in the layout of the C ABI (all arrays FP64, C order)."""

    n_core: int
    n_active: int
    n_virtual: int
    n_aux: int
    eps: np.ndarray              # [N]
    B: np.ndarray                # [M][N][N]
    gamma1: Optional[np.ndarray]  # [2][nA][nA]
    gamma2: Optional[np.ndarray]  # [3][nA]*4
    gamma3: Optional[np.ndarray]  # [4][nA]*6
    s: float
    ci: Optional[np.ndarray] = None   # [n_alpha_strings][n_beta_strings]
    n_alpha: int = 0                  # active alpha electrons
    n_beta: int = 0                   # active beta electrons
    name: str = ""
    f_offdiag: Optional[np.ndarray] = None   # [N][N] inter-block Fock elements, or None (zero)
    e0: float = 0.0                          # reference energy, only added to the total

    @property
    def N(self) -> int:
        return self.n_core + self.n_active + self.n_virtual

    @property
    def n_hole(self) -> int:
        return self.n_core + self.n_active

    @property
    def n_particle(self) -> int:
        return self.n_active + self.n_virtual

    def with_s(self, s: float) -> "Problem":
        return dataclasses.replace(self, s=float(s))

    def scaled(self, kappa: float) -> "Problem":
        """Same problem with B -> kappa * B (two-electron integrals scale by kappa^2)."""
        return dataclasses.replace(self, B=self.B * kappa)


# ---------------------------------------------------------------------------
# Fock-space helpers for the active space (input generation only)
# ---------------------------------------------------------------------------

def det_strings(n_orb: int, n_el: int) -> List[tuple]:
    """All occupation strings of n_el electrons in n_orb orbitals, lexicographic order."""
    return list(itertools.combinations(range(n_orb), n_el))


def _popcount_below(states: np.ndarray, k: int) -> np.ndarray:
    mask = np.uint64((1 << k) - 1)
    x = states & mask
    # vectorised popcount
    cnt = np.zeros(states.shape, dtype=np.int64)
    while np.any(x):
        cnt += (x & np.uint64(1)).astype(np.int64)
        x = x >> np.uint64(1)
    return cnt


class _Fock:
    """Dense Fock-space vectors over n_so spin orbitals (n_so <= 20)."""

    def __init__(self, n_so: int):
        if n_so > 20:
            raise ValueError("active Fock space limited to 20 spin orbitals")
        self.n_so = n_so
        self.dim = 1 << n_so
        self.states = np.arange(self.dim, dtype=np.uint64)
        self._sign = []
        for k in range(n_so):
            par = _popcount_below(self.states, k) & 1
            self._sign.append(np.where(par == 1, -1.0, 1.0))

    def annihilate(self, k: int, vec: np.ndarray) -> np.ndarray:
        """a_k acting on one or many vectors (last axis = Fock index)."""
        bit = np.uint64(1 << k)
        occ = (self.states & bit) != 0
        src = self.states[occ]
        dst = (src ^ bit).astype(np.int64)
        out = np.zeros_like(vec)
        out[..., dst] = vec[..., src.astype(np.int64)] * self._sign[k][occ]
        return out


def _ci_to_fock(ci: np.ndarray, n_orb: int, n_alpha: int, n_beta: int,
                fock: _Fock, alpha_offset: int, beta_offset: int) -> np.ndarray:
    a_str = det_strings(n_orb, n_alpha)
    b_str = det_strings(n_orb, n_beta)
    vec = np.zeros(fock.dim)
    for ia, sa in enumerate(a_str):
        ma = sum(1 << (alpha_offset + o) for o in sa)
        for ib, sb in enumerate(b_str):
            mb = sum(1 << (beta_offset + o) for o in sb)
            vec[ma | mb] = ci[ia, ib]
    return vec


def fock_rdms(vec: np.ndarray, fock: _Fock, order: int) -> np.ndarray:
    """Spin-orbital RDM of the given order from a Fock-space vector.

    Returns G with G[p1..pk, q1..qk] = <a+_p1 ... a+_pk a_qk ... a_q1>, computed as the
    Gram matrix of the k-fold annihilated vectors and expanded by antisymmetry.
    """
    n = fock.n_so
    tuples = list(itertools.combinations(range(n), order))
    if not tuples:                      # fewer spin orbitals than the order: zero density
        return np.zeros((n,) * (2 * order))
    # w_T = a_{t_k} ... a_{t_1} |psi>  for T = (t_1 < ... < t_k)
    W = np.empty((len(tuples), fock.dim))
    for idx, T in enumerate(tuples):
        w = vec
        for t in T:          # apply a_{t_1} first, then a_{t_2}, ...
            w = fock.annihilate(t, w)
        W[idx] = w
    # <w_P | w_Q> = <psi| a+_{p1} .. a+_{pk} a_{qk} .. a_{q1} |psi>
    gram = W @ W.T
    G = np.zeros((n,) * (2 * order))
    perms = list(itertools.permutations(range(order)))
    signs = []
    for pm in perms:
        inv = sum(1 for i in range(order) for j in range(i + 1, order) if pm[i] > pm[j])
        signs.append(-1.0 if inv % 2 else 1.0)
    tup = np.array(tuples, dtype=np.int64)           # [T][k]
    for pu, su in zip(perms, signs):
        up = tup[:, list(pu)]
        for pl, sl in zip(perms, signs):
            lo = tup[:, list(pl)]
            idx_up = tuple(up[:, i][:, None] for i in range(order))
            idx_lo = tuple(lo[:, i][None, :] for i in range(order))
            G[idx_up + idx_lo] = su * sl * gram
    return G


def random_ci(rng: np.random.Generator, n_orb: int, n_alpha: int, n_beta: int) -> np.ndarray:
    """i.i.d. N(0,1) coefficients over (alpha string x beta string), L2-normalised."""
    na = math.comb(n_orb, n_alpha)
    nb = math.comb(n_orb, n_beta)
    c = rng.standard_normal(na * nb).reshape(na, nb)
    return c / np.linalg.norm(c)


def active_rdms(ci: np.ndarray, n_orb: int, n_alpha: int, n_beta: int):
    """gamma1 [2][n]^2, gamma2 [3][n]^4, gamma3 [4][n]^6 of a CAS vector (spin-block layout).

    Per spin block (k indices, m of them alpha): the vectors w_T = a_{t_k} .. a_{t_1}|psi>
    of the index tuples T (m alpha then k - m beta orbitals, each part ascending) are
    gathered from the CI matrix with the signs of the annihilations; the block of sorted
    tuples is their Gram matrix, <w_P|w_Q> = <psi| a+_{p_1} .. a+_{p_k} a_{q_k} .. a_{q_1} |psi>,
    spread over all index orders with the permutation signs.  Strings only (no Fock space),
    so active spaces up to about 12 orbitals are generated in seconds."""
    n = n_orb
    c = np.asarray(ci, dtype=np.float64)
    out = []
    for k in (1, 2, 3):
        blocks = []
        for m in range(k, -1, -1):                       # alpha-first block order
            blocks.append(_rdm_block(c, n, n_alpha, n_beta, k, m))
        out.append(np.ascontiguousarray(np.stack(blocks)))
    return out[0], out[1], out[2]


def _annihilation_map(n: int, n_el: int, orbs):
    """a_{o_last} .. a_{o_first} on the strings of n_el electrons: for every string of
    n_el - len(orbs) electrons, the index of the source string (0 where none) and the sign
    (0 where none)."""
    src = {sum(1 << o for o in t): i for i, t in enumerate(itertools.combinations(range(n), n_el))}
    tm = sum(1 << o for o in orbs)
    tgt = list(itertools.combinations(range(n), n_el - len(orbs)))
    idx = np.zeros(len(tgt), dtype=np.int64)
    sgn = np.zeros(len(tgt))
    for j, t in enumerate(tgt):
        m = sum(1 << o for o in t)
        if m & tm:
            continue
        cur, sign = m | tm, 1.0
        for o in orbs:                                   # a_{orbs[0]} acts first
            if bin(cur & ((1 << o) - 1)).count("1") & 1:
                sign = -sign
            cur ^= 1 << o
        idx[j] = src[m | tm]
        sgn[j] = sign
    return idx, sgn


def _tuple_positions(n: int, r: int):
    """For every r-tuple of orbitals (row-major over [n]^r): its sorted combination's index
    in lexicographic order (-1 if an orbital repeats) and the sign of the sorting."""
    combos = {t: i for i, t in enumerate(itertools.combinations(range(n), r))}
    pos = np.full(n ** r, -1, dtype=np.int64)
    sgn = np.zeros(n ** r)
    for flat, t in enumerate(itertools.product(range(n), repeat=r)):
        if len(set(t)) < r:
            continue
        inv = sum(1 for i in range(r) for j in range(i + 1, r) if t[i] > t[j])
        pos[flat] = combos[tuple(sorted(t))]
        sgn[flat] = -1.0 if inv % 2 else 1.0
    return pos, sgn


def _rdm_block(c: np.ndarray, n: int, na: int, nb: int, k: int, m: int) -> np.ndarray:
    """Spin block of the k-body density with m alpha indices, [n]^(2k)."""
    shape = (n,) * (2 * k)
    Ta = list(itertools.combinations(range(n), m))
    Tb = list(itertools.combinations(range(n), k - m))
    if na - m < 0 or nb - (k - m) < 0 or not Ta or not Tb:
        return np.zeros(shape)
    amaps = [_annihilation_map(n, na, t) for t in Ta]
    bmaps = [_annihilation_map(n, nb, t) for t in Tb]
    # each beta annihilation passes the na - m alpha electrons left
    gsign = -1.0 if ((na - m) * (k - m)) % 2 else 1.0
    nra, nrb = len(amaps[0][0]), len(bmaps[0][0])
    W = np.empty((len(Ta), len(Tb), nra, nrb))
    for ia, (ida, sga) in enumerate(amaps):
        rows = c[ida] * sga[:, None]
        for ib, (idb, sgb) in enumerate(bmaps):
            W[ia, ib] = rows[:, idb] * (sgb * gsign)[None, :]
    W = W.reshape(len(Ta) * len(Tb), nra * nrb)
    G = W @ W.T                                          # sorted tuples (alpha part, beta part)
    pa, sa = _tuple_positions(n, m)
    pb, sb = _tuple_positions(n, k - m)
    # full index tuple = (alpha part, beta part), row-major
    pos = (pa[:, None] * len(Tb) + pb[None, :]).ravel()
    sgn = (sa[:, None] * sb[None, :]).ravel()
    valid = (pa[:, None] >= 0) & (pb[None, :] >= 0)
    pos = np.where(valid.ravel(), pos, 0)
    sgn = np.where(valid.ravel(), sgn, 0.0)
    out = sgn[:, None] * sgn[None, :] * G[np.ix_(pos, pos)]
    return out.reshape(shape)


# ---------------------------------------------------------------------------
# Problem generation
# ---------------------------------------------------------------------------

def _draw_B(rng: np.random.Generator, M: int, N: int, sigma: float = 0.1) -> np.ndarray:
    iu = np.triu_indices(N)
    vals = rng.standard_normal(M * len(iu[0])) * sigma
    B = np.zeros((M, N, N))
    vals = vals.reshape(M, len(iu[0]))
    B[:, iu[0], iu[1]] = vals
    B[:, iu[1], iu[0]] = vals
    return B


def make_problem(n_core: int, n_active: int, n_virtual: int, n_aux: int, seed: int,
                 s: float = 0.5, gap: float = 1.0, name: str = "",
                 with_gamma3: bool = True, f_sigma: float = 0.0,
                 n_alpha: Optional[int] = None, n_beta: Optional[int] = None) -> Problem:
    """Draw one problem.

    Draw order (part of the contract so both sides reproduce it): core energies,
    active energies, virtual energies, B, CI vector, then (only with f_sigma > 0) the
    inter-block Fock elements.  ``gap`` in (0, 1] scales the
    inner edges of the energy windows toward zero to mimic a stretched bond:
    core U(-2, -0.5 gap), active U(-0.3 gap, 0.3 gap), virtual U(0.2 gap, 3).
    ``f_sigma`` > 0 adds a symmetric f_offdiag with N(0, f_sigma^2) entries on the
    core-active, core-virtual and active-virtual blocks (upper triangle drawn row-major,
    mirrored) and zeros inside the blocks.  ``n_alpha``, ``n_beta`` (default
    ceil(nA/2), floor(nA/2)) set the electron numbers of the CAS vector, e.g. a few
    electrons in a large active space whose half-filled vector would be too long to draw.
    """
    rng = np.random.default_rng(seed)
    N = n_core + n_active + n_virtual
    ec = np.sort(rng.uniform(-2.0, -0.5 * gap, n_core))
    ea = np.sort(rng.uniform(-0.3 * gap, 0.3 * gap, n_active))
    ev = np.sort(rng.uniform(0.2 * gap, 3.0, n_virtual))
    eps = np.concatenate([ec, ea, ev])
    B = _draw_B(rng, n_aux, N)
    n_alpha = (n_active + 1) // 2 if n_alpha is None else int(n_alpha)
    n_beta = n_active // 2 if n_beta is None else int(n_beta)
    if n_active > 0:
        ci = random_ci(rng, n_active, n_alpha, n_beta)
        g1, g2, g3 = active_rdms(ci, n_active, n_alpha, n_beta)
        if not with_gamma3:
            g3 = None
    else:
        ci, g1, g2, g3 = None, None, None, None
    f = None
    if f_sigma > 0.0:
        blk = np.array([0] * n_core + [1] * n_active + [2] * n_virtual)
        iu = np.triu_indices(N, k=1)
        inter = blk[iu[0]] != blk[iu[1]]
        vals = rng.standard_normal(int(inter.sum())) * f_sigma
        f = np.zeros((N, N))
        f[iu[0][inter], iu[1][inter]] = vals
        f[iu[1][inter], iu[0][inter]] = vals
    return Problem(n_core, n_active, n_virtual, n_aux, eps, B, g1, g2, g3, float(s),
                   ci=ci, n_alpha=n_alpha, n_beta=n_beta, name=name, f_offdiag=f)


# The five workloads: shapes from the paper's CAS(2,2), CAS(6,6) and CAS(8,8)
# references, s = 0.5 and 1.0, dissociation curves, and the ~100-electron regime.
CONFIGS = {
    "tiny":   dict(n_core=2, n_active=2, n_virtual=10, n_aux=40, seed=101, s=0.5),
    "small":  dict(n_core=5, n_active=6, n_virtual=49, n_aux=200, seed=202, s=0.5),
    "medium": dict(n_core=20, n_active=8, n_virtual=300, n_aux=1200, seed=303, s=0.5),
    "large":  dict(n_core=43, n_active=2, n_virtual=185, n_aux=920, seed=505, s=0.5),
}
SMALL_S_VALUES = (0.1, 0.5, 1.0)


def make_config(name: str, s: Optional[float] = None) -> Problem:
    kw = dict(CONFIGS[name])
    if s is not None:
        kw["s"] = s
    return make_problem(name=name, **kw)


def make_batch_config(n_geom: int = 64, base_seed: int = 4000, s: float = 0.5,
                      first: int = 0) -> List[Problem]:
    """Uneven geometries along a synthetic dissociation curve.

    Geometry k draws its sizes first (core U{5..15}, active U{4..8}, virtual
    U{80..400}), then uses naux = 4 N and gap factor 1 - 0.8 k/63.
    """
    probs = []
    for k, (nc, na, nv) in zip(range(first, first + n_geom), batch_sizes(n_geom, base_seed, first)):
        N = nc + na + nv
        gap = 1.0 - 0.8 * k / 63.0
        probs.append(make_problem(nc, na, nv, 4 * N, seed=base_seed + 10000 + k, s=s,
                                  gap=gap, name=f"curve{k}"))
    return probs


def batch_sizes(n_geom: int = 64, base_seed: int = 4000, first: int = 0):
    """(n_core, n_active, n_virtual) of the curve geometries first .. first + n_geom - 1,
    without drawing their arrays."""
    out = []
    for k in range(first, first + n_geom):
        rng = np.random.default_rng(base_seed + k)
        nc = int(rng.integers(5, 16))
        na = int(rng.integers(4, 9))
        nv = int(rng.integers(80, 401))
        out.append((nc, na, nv))
    return out
