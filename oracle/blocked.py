"""The commutator engine of ``gno`` evaluated block by block (oracle level O2; FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

``gno`` holds every operator as a dense tensor over all 2N spin orbitals, which cannot
reach the medium and large workloads: their antisymmetrised integrals alone would need
(2N)^4 doubles.  This module runs the same algebra -- GNO -> bare conversion with the
reference densities, the bare commutator from the anticommutation relations only
(``gno.bare_commutator_terms``, shared as is), and the bare -> GNO projection with the
"1,2" truncation (Sec. II.A) -- on tensors stored as dense blocks over the six
spin-orbital blocks [core a, core b, active a, active b, virtual a, virtual b]:

* a zero block is simply absent, so the excitation-only amplitudes, the block-diagonal
  densities and the spin structure prune every product term before any arithmetic;
* the antisymmetrised integrals <pq||rs> are never stored: each block is built when a
  term needs it from the factorised tensor, (pq|rs) = sum_Q B^Q_pq B^Q_rs (Sec. III,
  Eq. int_fact), and a block too large for memory (the (VV|VV) type, Sec. III,
  Eq. scaling_problem) is built and consumed in batches of its first index;
* the reference densities enter through their cumulant expansions (two- and three-body
  densities as sums of products of gamma and the cumulants lambda2, lambda3), never as
  dense hole-space arrays.

Only the evaluation differs from ``gno``; the terms, signs and projections are the same,
and ``tests/test_oracle_df.py`` checks this level against ``gno``/``dsrg`` element by
element on micro and tiny inputs and against the stored small-workload values.

Parity: pinned to the generic engine (itself pinned in the full Fock space).
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .gno import Term, bare_commutator_terms

# orbital blocks in the oracle's spin-orbital order
SPACE = "CCAAVV"
SPIN = (0, 1, 0, 1, 0, 1)
SETS = dict(G=(0, 1, 2, 3, 4, 5), H=(0, 1, 2, 3), P=(2, 3, 4, 5), C=(0, 1), A=(2, 3), V=(4, 5))
# a lazily built block above this many doubles is produced in batches of its first index
BATCH_ELEMS = 1 << 26


class Orb:
    """Sizes and offsets of the six orbital blocks."""

    def __init__(self, nC: int, nA: int, nV: int):
        self.nC, self.nA, self.nV = nC, nA, nV
        self.n = (nC, nC, nA, nA, nV, nV)
        self.sp0 = (0, 0, nC, nC, nC + nA, nC + nA)          # first spatial orbital
        self.off = tuple(int(x) for x in np.cumsum((0,) + self.n)[:-1])   # spin-orbital offset
        self.N = nC + nA + nV

    def shape(self, key):
        return tuple(self.n[b] for b in key)

    def spatial(self, b, lo=0, hi=None):
        hi = self.n[b] if hi is None else hi
        return slice(self.sp0[b] + lo, self.sp0[b] + hi)


def spin_ok(key) -> bool:
    """A one- or two-body block conserves spin (upper and lower spins equal as multisets)."""
    k = len(key) // 2
    return sorted(SPIN[b] for b in key[:k]) == sorted(SPIN[b] for b in key[k:])


# ---------------------------------------------------------------------------
# tensors
# ---------------------------------------------------------------------------
class BT:
    """Explicit blocks: key (tuple of block indices) -> ndarray; absent keys are zero."""

    lazy = False

    def __init__(self, orb: Orb, rank: int, blocks: Optional[dict] = None):
        self.orb = orb
        self.rank = rank
        self.blocks = {} if blocks is None else blocks

    def has(self, key):
        return key in self.blocks

    def get(self, key, batch=None):
        a = self.blocks[key]
        if batch is not None:
            ax, lo, hi = batch
            a = a[(slice(None),) * ax + (slice(lo, hi),)]
        return a

    def add(self, key, arr, out_slice=None):
        if key not in self.blocks:
            self.blocks[key] = np.zeros(self.orb.shape(key))
        if out_slice is None:
            self.blocks[key] += arr
        else:
            self.blocks[key][out_slice] += arr

    @classmethod
    def from_dense(cls, orb: Orb, dense: np.ndarray, sets: Sequence[str], base: int = 0):
        """Blocks of a dense array whose axis k spans the blocks SETS[sets[k]] contiguously,
        starting at spin-orbital offset ``base`` for the first of them; all-zero blocks dropped."""
        t = cls(orb, dense.ndim)
        starts = []
        for s in sets:
            st, o = {}, 0
            for b in SETS[s]:
                st[b] = o
                o += orb.n[b]
            starts.append(st)
        for key in itertools.product(*[SETS[s] for s in sets]):
            if any(orb.n[b] == 0 for b in key):
                continue
            sl = tuple(slice(starts[k][b], starts[k][b] + orb.n[b]) for k, b in enumerate(key))
            blk = dense[sl]
            if np.any(blk != 0.0):
                t.blocks[key] = np.array(blk)
        return t

    def to_dense(self, sets: Sequence[str]) -> np.ndarray:
        dims, starts = [], []
        for s in sets:
            st, o = {}, 0
            for b in SETS[s]:
                st[b] = o
                o += self.orb.n[b]
            dims.append(o)
            starts.append(st)
        out = np.zeros(dims)
        for key, blk in self.blocks.items():
            if all(b in starts[k] for k, b in enumerate(key)):
                sl = tuple(slice(starts[k][b], starts[k][b] + self.orb.n[b]) for k, b in enumerate(key))
                out[sl] += blk
        return out


class DFV:
    """Antisymmetrised integrals <pq||rs> = (pr|qs) d(sp,sr) d(sq,ss) - (ps|qr) d(sp,ss) d(sq,sr)
    (C-convention, coefficient of 1/4 {a+_p a+_q a_s a_r}), every block assembled on demand
    from Coulomb blocks (pr|qs) = sum_Q B^Q_pr B^Q_qs over the spatial core, active and
    virtual ranges (Eq. int_fact).  Coulomb blocks up to ``keep_elems`` doubles are kept once
    built (a budget of ``cache_elems`` in all); larger ones are built for each use, and
    consumed in batches of one index when above BATCH_ELEMS."""

    lazy = True
    rank = 4

    def __init__(self, orb: Orb, B: np.ndarray, cache_elems: int = 1 << 30, keep_elems: int = 1 << 27,
                 piece_elems: int = 3 * BATCH_ELEMS):
        self.orb = orb
        self.B = B
        self._keys = None
        self.cache = {}
        self.cache_left = cache_elems
        self.keep_elems = keep_elems
        # the most recent pieces of batched builds (first in, first out), so that the
        # products queued on one batch range share each piece
        self.pieces = {}
        self.piece_elems = piece_elems

    def has(self, key):
        if any(self.orb.n[b] == 0 for b in key):
            return False
        p, q, r, s = (SPIN[b] for b in key)
        return (p == r and q == s) or (p == s and q == r)

    def elems(self, key):
        return int(np.prod(self.orb.shape(key)))

    def _coulomb(self, rp, rr, rq, rs, keep=True):
        """(pr|qs) over four spatial ranges (start, stop), as an array [p][r][q][s]."""
        key = (rp, rr, rq, rs)
        hit = self.cache.get(key)
        if hit is None:
            hit = self.pieces.get(key)
        if hit is not None:
            return hit
        B = self.B
        n1 = (rp[1] - rp[0]) * (rr[1] - rr[0])
        n2 = (rq[1] - rq[0]) * (rs[1] - rs[0])
        X = B[:, rp[0]:rp[1], rr[0]:rr[1]].reshape(B.shape[0], n1)
        Y = B[:, rq[0]:rq[1], rs[0]:rs[1]].reshape(B.shape[0], n2)
        J = (X.T @ Y).reshape(rp[1] - rp[0], rr[1] - rr[0], rq[1] - rq[0], rs[1] - rs[0])
        if keep and J.size <= self.keep_elems and J.size <= self.cache_left:
            self.cache[key] = J
            self.cache_left -= J.size
        elif not keep:
            self.pieces[key] = J
            while sum(x.size for x in self.pieces.values()) > self.piece_elems and len(self.pieces) > 1:
                del self.pieces[next(iter(self.pieces))]
        return J

    def get(self, key, batch=None):
        """Block ``key``; batch = (axis, lo, hi) restricts that axis to [lo, hi)."""
        o = self.orb
        bp, bq, br, bs = key
        rng = [(o.sp0[b], o.sp0[b] + o.n[b]) for b in key]
        if batch is not None:
            ax, lo, hi = batch
            b = key[ax]
            rng[ax] = (o.sp0[b] + lo, o.sp0[b] + hi)
        P, Q, R, S = rng
        out = None
        if SPIN[bp] == SPIN[br] and SPIN[bq] == SPIN[bs]:
            out = self._coulomb(P, R, Q, S, batch is None).transpose(0, 2, 1, 3)   # (pr|qs) at [p,q,r,s]
        if SPIN[bp] == SPIN[bs] and SPIN[bq] == SPIN[br]:
            x = self._coulomb(P, S, Q, R, batch is None).transpose(0, 2, 3, 1)     # (ps|qr) at [p,q,r,s]
            out = -x if out is None else out - x
        return out


class View:
    """coef * base transposed: view[i_0 .. i_k] = coef * base[...] with view axis k equal to
    base axis axes[k] (numpy transpose semantics); shares the base's storage."""

    def __init__(self, base, axes=None, coef: float = 1.0):
        self.base = base
        self.rank = base.rank
        self.axes = tuple(range(base.rank)) if axes is None else tuple(axes)
        self.coef = coef
        self.lazy = base.lazy

    def _bkey(self, key):
        bk = [None] * self.rank
        for k, a in enumerate(self.axes):
            bk[a] = key[k]
        return tuple(bk)

    def has(self, key):
        return self.base.has(self._bkey(key))

    def elems(self, key):
        return int(np.prod(self.base.orb.shape(key)))

    def batch_axis(self):
        """the view axis of the base's first axis (batched first for lazy bases)."""
        return self.axes.index(0)

    def get(self, key, batch=None):
        bb = None
        if batch is not None:
            bb = (self.axes[batch[0]], batch[1], batch[2])
        return self.base.get(self._bkey(key), bb).transpose(self.axes)


def view(t, axes=None, coef=1.0):
    if isinstance(t, Sum):
        return Sum([view(p, axes, coef) for p in t.parts])
    if isinstance(t, View):
        ax = tuple(range(t.rank)) if axes is None else tuple(axes)
        return View(t.base, tuple(t.axes[a] for a in ax), t.coef * coef)
    return View(t, axes, coef)


class Sum:
    """A sum of tensors of one rank (expanded term by term by the evaluator)."""

    def __init__(self, parts):
        self.parts = [p for p in parts if p is not None]
        self.rank = self.parts[0].rank


def parts_of(t):
    """(coef, plain tensor) alternatives of a factor."""
    if t is None:
        return []
    if isinstance(t, Sum):
        out = []
        for p in t.parts:
            out.extend(parts_of(p))
        return out
    if isinstance(t, View):
        return [(t.coef, t)]
    return [(1.0, t)]


class Product:
    """A factor given as a sum of products: alternatives [(coef, [(tensor, letters), ...])]
    over the letters of the factor it replaces (the cumulant expansions of the densities)."""

    def __init__(self, alts):
        self.alts = alts


# ---------------------------------------------------------------------------
# block evaluation of product terms
# ---------------------------------------------------------------------------
def _elems(t, key, orb):
    return int(np.prod(orb.shape(key)))


def beval(orb: Orb, terms: Sequence[Term], out_letters: str, ranges: Dict[str, Sequence[int]],
          rename: Optional[Dict[str, str]] = None, extra=(), sign: float = 1.0, out=None):
    """sum over terms of coef * prod factors (letters renamed, extra factors appended),
    every letter over the blocks ranges[letter] (default: all), into ``out`` (a BT of rank
    len(out_letters)) or, for out_letters == "", returned as a float."""
    rename = rename or {}
    scalar = out_letters == ""
    total = 0.0
    deferred = []
    if out is None and not scalar:
        out = BT(orb, len(out_letters))
    for t in terms:
        facs = []
        for (T, lets) in t.factors:
            facs.append((T, "".join(rename.get(l, l) for l in lets)))
        # expand sums and products into plain alternatives
        alts = [(t.coef * sign, [])]
        for (T, lets) in list(facs) + list(extra):
            if isinstance(T, Product):
                new = []
                for c0, fl in alts:
                    for c1, pl in T.alts:
                        new.append((c0 * c1, fl + list(pl)))
                alts = new
                continue
            ps = parts_of(T)
            new = []
            for c0, fl in alts:
                for c1, p in ps:
                    new.append((c0 * c1, fl + [(p, lets)]))
            alts = new
        for coef, fl in alts:
            if coef == 0.0 or not fl:
                continue
            total += _eval_product(orb, coef, fl, out_letters, ranges, out, deferred)
    total += _run_batched(deferred, out_letters, out)
    return total if scalar else out


def _eval_product(orb, coef, fl, out_letters, ranges, out, deferred):
    letters = set()
    for _, lets in fl:
        letters.update(lets)
    for l in out_letters:
        if l not in letters:
            raise ValueError("output letter %s not in the product" % l)
    total = 0.0
    for asg in _assignments(orb, fl, ranges):
        total += _contract(orb, coef, fl, out_letters, asg, out, deferred)
    return total


def _assignments(orb, fl, ranges):
    """Every assignment of orbital blocks to the letters of a product under which all its
    factors have a non-zero block: a join over the factors' key sets, most selective
    factor first."""
    facs = []
    for T, lets in fl:
        allowed = [set(b for b in ranges.get(l, SETS["G"]) if orb.n[b] > 0) for l in lets]
        ks = [k for k in keyset(T, orb) if all(b in al for b, al in zip(k, allowed))]
        if not ks:
            return []
        facs.append((ks, lets))
    facs.sort(key=lambda f: len(f[0]))
    asgs = [dict()]
    for ks, lets in facs:
        done = [i for i, l in enumerate(lets) if l in asgs[0]]
        index = {}
        for k in ks:
            index.setdefault(tuple(k[i] for i in done), []).append(k)
        new = []
        for a in asgs:
            for k in index.get(tuple(a[lets[i]] for i in done), ()):
                b = dict(a)
                ok = True
                for l, blk in zip(lets, k):
                    if b.setdefault(l, blk) != blk:
                        ok = False
                        break
                if ok:
                    new.append(b)
        asgs = new
        if not asgs:
            return []
    return asgs


def keyset(T, orb):
    """The keys of the non-zero blocks of a factor (a set, for the pruning of the block
    assignments)."""
    if isinstance(T, BT):
        return set(T.blocks)
    if isinstance(T, View):
        base = keyset(T.base, orb)
        return {tuple(k[a] for a in T.axes) for k in base}
    if isinstance(T, DFV):
        if T._keys is None:
            T._keys = {k for k in itertools.product(range(6), repeat=4) if T.has(k)}
        return T._keys
    raise TypeError(type(T))


_PATHS = {}


def _einsum(spec, arrs):
    """np.einsum: direct summation when the product of all index ranges is small, else the
    pairwise (BLAS) order computed once per (spec, shapes)."""
    key = (spec,) + tuple(a.shape for a in arrs)
    path = _PATHS.get(key)
    if path is None:
        dims = {}
        for lets, a in zip(spec.split("->")[0].split(","), arrs):
            for l, n in zip(lets, a.shape):
                dims[l] = n
        naive = float(np.prod([float(n) for n in dims.values()])) if dims else 1.0
        path = False if naive <= 4096 else np.einsum_path(spec, *arrs, optimize="greedy")[0]
        _PATHS[key] = path
    if path is False:
        return np.einsum(spec, *arrs)
    return np.einsum(spec, *arrs, optimize=path)


def _big_factor(orb, fl, keys):
    """The lazily built factor block too large to build whole (the largest), or None."""
    big = None
    for (T, lets), key in zip(fl, keys):
        if getattr(T, "lazy", False) and T.elems(key) > BATCH_ELEMS:
            if big is None or T.elems(key) > big[2]:
                big = (T, lets, T.elems(key), key)
    return big


def _contract(orb, coef, fl, out_letters, asg, out, deferred):
    """One product under one block assignment: contracted at once, or (when a lazily built
    factor is too large) queued in ``deferred`` for the batched pass of ``_run_batched``."""
    keys = [tuple(asg[l] for l in lets) for (_, lets) in fl]
    big = _big_factor(orb, fl, keys)
    spec = ",".join(lets for (_, lets) in fl) + "->" + out_letters
    okey = tuple(asg[l] for l in out_letters)
    if big is None:
        arrs = [T.get(k) for (T, _), k in zip(fl, keys)]
        val = _einsum(spec, arrs) * coef
        if out is None:
            return float(val)
        out.add(okey, val)
        return 0.0
    T, lets, n, key = big
    ax = T.batch_axis() if isinstance(T, View) else 0
    bl = lets[ax]
    nb = orb.n[asg[bl]]
    step = max(1, int(BATCH_ELEMS * nb // n))
    deferred.append((nb, step, coef, fl, keys, spec, okey, bl))
    return 0.0


def _run_batched(deferred, out_letters, out):
    """The queued products, batch range outermost: every product that reads the same lazily
    built block in the same batches runs on one build of each batch piece (the lazy
    tensors keep the pieces of the current range)."""
    total = 0.0
    groups = {}
    for task in deferred:
        groups.setdefault(task[:2], []).append(task)
    for (nb, step), tasks in groups.items():
        for lo in range(0, nb, step):
            hi = min(nb, lo + step)
            for (_, _, coef, fl, keys, spec, okey, bl) in tasks:
                arrs = []
                for (Tf, lf), k in zip(fl, keys):
                    if bl in lf:
                        a_ = lf.index(bl)
                        if getattr(Tf, "lazy", False):
                            arrs.append(Tf.get(k, (a_, lo, hi)))
                        else:
                            arrs.append(Tf.get(k)[(slice(None),) * a_ + (slice(lo, hi),)])
                    else:
                        arrs.append(Tf.get(k))
                val = _einsum(spec, arrs) * coef
                if out is None:
                    total += float(val)
                elif bl in out_letters:
                    a_ = out_letters.index(bl)
                    out.add(okey, val, (slice(None),) * a_ + (slice(lo, hi),))
                else:
                    out.add(okey, val)
    return total


# ---------------------------------------------------------------------------
# reference densities in block form (cumulant expansions)
# ---------------------------------------------------------------------------
class BlockDensities:
    """gamma (1 on core, the input on active), lambda2, lambda3 over the active blocks, and
    the plain-order two- and three-body densities over the hole space as sums of products
    (the cumulant expansion of Sec. II.A): no hole-space array of rank above 2 is formed."""

    def __init__(self, orb: Orb, gA: np.ndarray, L2a: np.ndarray, L3a: np.ndarray):
        self.orb = orb
        g = BT(orb, 2)
        for b in SETS["C"]:
            if orb.n[b]:
                g.blocks[(b, b)] = np.eye(orb.n[b])
        if orb.nA:
            nA = orb.nA
            for b, s in ((2, 0), (3, 1)):
                g.blocks[(b, b)] = np.array(gA[s * nA:(s + 1) * nA, s * nA:(s + 1) * nA])
        self.gamma = g
        self.L2 = BT.from_dense(orb, L2a, "AAAA") if orb.nA else BT(orb, 4)
        self.L3 = BT.from_dense(orb, L3a, "AAAAAA") if (orb.nA and L3a is not None) else BT(orb, 6)

    def D2p(self, m, n, o, q):
        """<a+_m a+_n a_o a_q> = g[m,q] g[n,o] - g[m,o] g[n,q] + lambda2^{mn}_{qo}."""
        g = self.gamma
        return Product([(1.0, [(g, m + q), (g, n + o)]), (-1.0, [(g, m + o), (g, n + q)]),
                        (1.0, [(self.L2, m + n + q + o)])])

    def D3p(self, a, b, c, d, e, f):
        """<a+_a a+_b a+_c a_d a_e a_f> = G3[a,b,c,f,e,d] with the C-convention three-body
        density G3 = det(g g g) + antisymmetrised g x lambda2 + lambda3."""
        g = self.gamma
        up, lo = (a, b, c), (f, e, d)
        alts = []
        for pm in itertools.permutations(range(3)):
            inv = sum(1 for i in range(3) for j in range(i + 1, 3) if pm[i] > pm[j])
            alts.append((-1.0 if inv % 2 else 1.0,
                         [(g, up[0] + lo[pm[0]]), (g, up[1] + lo[pm[1]]), (g, up[2] + lo[pm[2]])]))
        for i in range(3):
            for j in range(3):
                ru = [up[k] for k in range(3) if k != i]
                rl = [lo[k] for k in range(3) if k != j]
                alts.append(((-1.0) ** (i + j), [(g, up[i] + lo[j]), (self.L2, "".join(ru + rl))]))
        alts.append((1.0, [(self.L3, "".join(up + lo))]))
        return Product(alts)


# ---------------------------------------------------------------------------
# the engine of gno, block by block
# ---------------------------------------------------------------------------
def gno_to_bare(orb: Orb, op, dens: BlockDensities):
    """(k0, K1, K2) in MK-GNO form (plain order) -> the same operator in true-vacuum order
    (as ``gno.gno_to_bare``): one-body gains the single contractions of K2 with gamma over
    the holes, the constant the full contractions."""
    k0, K1, K2 = op
    H = SETS["H"]
    g = dens.gamma
    B1 = BT(orb, 2)
    if K1 is not None:
        beval(orb, [Term(1.0, [(K1, "xy")], "xy")], "xy", {}, out=B1)
    b0 = k0
    if K1 is not None:
        b0 -= beval(orb, [Term(1.0, [(K1, "pq"), (g, "pq")], "")], "", dict(p=H, q=H))
    if K2 is not None:
        rng = dict(p=H, q=H, r=H, s=H)
        beval(orb, [Term(1.0, [(K2, "pxry"), (g, "pr")], "xy"), Term(-1.0, [(K2, "pxys"), (g, "ps")], "xy"),
                    Term(-1.0, [(K2, "xqry"), (g, "qr")], "xy"), Term(1.0, [(K2, "xqys"), (g, "qs")], "xy")],
              "xy", rng, out=B1)
        b0 += 2.0 * beval(orb, [Term(1.0, [(K2, "pqrs"), (g, "ps"), (g, "qr")], ""),
                                Term(-1.0, [(K2, "pqrs"), (g, "pr"), (g, "qs")], "")], "", rng)
        b0 -= beval(orb, [Term(1.0, [(K2, "pqrs")], "")], "", rng, extra=[(dens.D2p("p", "q", "r", "s"), "")])
    return (b0, B1, K2)


def _project(orb: Orb, R1, R2, R3, dens: BlockDensities, want0: bool, want1, want2):
    """GNO scalar, one-body block want1 = (sets of c, d) and two-body block want2 of the bare
    operator R1 + R2 + R3 (plain order), as ``gno._project``."""
    H = SETS["H"]
    g = dens.gamma
    out0, out1, out2 = 0.0, None, None
    if want2 is not None:
        rc1, rc2, rd1, rd2 = (SETS[x] for x in want2)
        out2 = BT(orb, 4)
        beval(orb, R2, "abcd", dict(a=rc1, b=rc2, c=rd1, d=rd2), out=out2)
        cre, ann = "abc", "def"
        for i in range(3):
            for j in range(3):
                ci, dj = cre[i], ann[j]
                rest_c = [x for x in cre if x != ci]
                rest_a = [x for x in ann if x != dj]
                ren = {rest_c[0]: "w", rest_c[1]: "x", rest_a[0]: "y", rest_a[1]: "z", ci: "m", dj: "n"}
                rng = dict(w=rc1, x=rc2, y=rd1, z=rd2, m=H, n=H)
                beval(orb, R3, "wxyz", rng, rename=ren, extra=[(g, "mn")], sign=(-1.0) ** (i + j), out=out2)
    if want1 is not None:
        rc, rd = (SETS[x] for x in want1)
        out1 = BT(orb, 2)
        beval(orb, R1, "cd", dict(c=rc, d=rd), rename={"a": "c", "b": "d"}, out=out1)
        for (ci, dj, sgn) in (("a", "c", -1.0), ("a", "d", 1.0), ("b", "c", 1.0), ("b", "d", -1.0)):
            rc_ = [x for x in "ab" if x != ci][0]
            ra_ = [x for x in "cd" if x != dj][0]
            ren = {rc_: "x", ra_: "y", ci: "m", dj: "n"}
            beval(orb, R2, "xy", dict(x=rc, y=rd, m=H, n=H), rename=ren, extra=[(g, "mn")], sign=sgn, out=out1)
        cre, ann = "abc", "def"
        for (i1, i2) in itertools.combinations(range(3), 2):
            for (j1, j2) in itertools.combinations(range(3), 2):
                k = [x for x in range(3) if x not in (i1, i2)][0]
                l = [x for x in range(3) if x not in (j1, j2)][0]
                ren = {cre[i1]: "m", cre[i2]: "n", ann[j1]: "o", ann[j2]: "q", cre[k]: "x", ann[l]: "y"}
                sgn = (-1.0) ** ((i1 + 1) + (i2 + 1) + (j1 + 1) + (j2 + 1))
                beval(orb, R3, "xy", dict(x=rc, y=rd, m=H, n=H, o=H, q=H), rename=ren,
                      extra=[(dens.D2p("m", "n", "o", "q"), "")], sign=sgn, out=out1)
    if want0:
        out0 += beval(orb, R1, "", dict(c=H, d=H), rename={"a": "c", "b": "d"}, extra=[(g, "cd")])
        out0 += beval(orb, R2, "", dict(a=H, b=H, c=H, d=H), extra=[(dens.D2p("a", "b", "c", "d"), "")])
        if R3:
            out0 += beval(orb, R3, "", {k: H for k in "abcdef"},
                          extra=[(dens.D3p("a", "b", "c", "d", "e", "f"), "")])
    return out0, out1, out2


def commutator(orb: Orb, X, Y, dens: BlockDensities, want0=False, want1=None, want2=None):
    """GNO parts of [X, Y]_{1,2} (plain-order GNO operators), as ``gno.commutator``; the
    requested blocks are named by space letters, e.g. want2 = "PPHH"."""
    Xb = gno_to_bare(orb, X, dens)
    Yb = gno_to_bare(orb, Y, dens)
    R1, R2, R3 = bare_commutator_terms(Xb, Yb)
    return _project(orb, R1, R2, R3, dens, want0, want1, want2)
