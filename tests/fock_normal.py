"""Normal products of the Mukherjee-Kutzelnigg generalised normal order (Sec. II.A) as
operators in the full Fock space, built from brute-force reference expectation values
(no cumulant or density code of the oracle): test helpers."""
from __future__ import annotations

import itertools


def fock_string(fs, cre, ann, vec):
    """a+_{c1} .. a+_{ck} a_{d1} .. a_{dk} |vec> (bare plain-order string)."""
    w = vec
    for d in reversed(ann):
        w = fs.ann[d] @ w
    for c in reversed(cre):
        w = fs.cre[c] @ w
    return w


def normal_product_action(fs, psi0, cre, ann, vec, memo):
    """{a+_{c1} .. a+_{ck} a_{d1} .. a_{dk}} |vec> for the multideterminantal reference psi0
    (Mukherjee-Kutzelnigg generalised normal order, Sec. II.A), built recursively in the
    full Fock space:
        bare string = sum over equal-size subsets I of creators and J of annihilators of
                      sign(I, J) <psi0| removed string |psi0> {remaining string},
    where the I = J = {} term is the normal product itself and the expectation values are
    brute-force matrix elements of psi0 (no cumulant or density code of the oracle)."""
    key = (tuple(cre), tuple(ann))
    if key in memo:
        return memo[key]
    k = len(cre)
    out = fock_string(fs, cre, ann, vec)
    if k > 0:
        for m in range(1, k + 1):
            for I in itertools.combinations(range(k), m):
                for J in itertools.combinations(range(k), m):
                    removed = [i for i in I] + [k + j for j in J]
                    rest = [i for i in range(2 * k) if i not in removed]
                    # sign of the permutation (removed block first, order kept in each block)
                    perm = removed + rest
                    sgn = perm_sign_local(perm)
                    rc = [cre[i] for i in I]
                    ra = [ann[j] for j in J]
                    dens = psi0 @ fock_string(fs, rc, ra, psi0)
                    if dens == 0.0:
                        continue
                    kc = [cre[i] for i in range(k) if i not in I]
                    ka = [ann[j] for j in range(k) if j not in J]
                    out = out - sgn * dens * normal_product_action(fs, psi0, kc, ka, vec, memo)
    memo[key] = out
    return out


def perm_sign_local(perm):
    inv = sum(1 for i in range(len(perm)) for j in range(i + 1, len(perm)) if perm[i] > perm[j])
    return -1.0 if inv % 2 else 1.0
