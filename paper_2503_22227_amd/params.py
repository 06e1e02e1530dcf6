"""Parameter derivation for the library: NTT-friendly prime chains.

The primes of a chain are chosen as follows (a reading: the paper fixes only
N, the number of limbs and the total modulus size of its benchmark chain):
every prime is 1 mod 2*N_max, primes of one bit size are taken from the
largest downwards, the chain's size list is consumed in order (Q primes, then
special primes, then auxiliary bases) and no prime is used twice.  The library
computes its roots of unity and every other table from these primes itself.
"""
from __future__ import annotations

from typing import Dict, List


def _probable_prime(n: int) -> bool:
    """Miller-Rabin with the first twelve prime bases: exact below 3.3e24."""
    if n < 2:
        return False
    witnesses = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37]
    if n in witnesses:
        return True
    if any(n % w == 0 for w in witnesses):
        return False
    s = (n - 1 & -(n - 1)).bit_length() - 1
    d = (n - 1) >> s
    for w in witnesses:
        y = pow(w, d, n)
        if y == 1 or y == n - 1:
            continue
        for _ in range(s - 1):
            y = pow(y, 2, n)
            if y == n - 1:
                break
        else:
            return False
    return True


def prime_chain(size_groups: List[List[int]], two_nmax: int) -> List[List[int]]:
    """Primes for each group of bit sizes; a prime of b bits is the largest unused
    prime = 1 mod two_nmax below 2^b."""
    taken = set()
    cursor: Dict[int, int] = {}
    out = []
    for group in size_groups:
        primes = []
        for bits in group:
            c = cursor.get(bits)
            if c is None:
                c = (((1 << bits) - 1) // two_nmax) * two_nmax + 1
                if c >= (1 << bits):
                    c -= two_nmax
            while not (c not in taken and _probable_prime(c)):
                c -= two_nmax
                if c < (1 << (bits - 1)):
                    raise ValueError("no %d-bit NTT-friendly prime left" % bits)
            taken.add(c)
            primes.append(c)
            cursor[bits] = c - two_nmax
        out.append(primes)
    return out


def chain_for(workload: dict) -> dict:
    """Prime lists of a workload description: {'q': [...], 'p': [...], 'b': [...], 'msk': int}."""
    groups = [workload["q_bits"], workload["p_bits"]]
    if workload.get("b_bits"):
        groups += [workload["b_bits"], [workload["msk_bits"]]]
    ch = prime_chain(groups, 2 << workload["log_nmax"])
    return {"q": ch[0], "p": ch[1], "b": ch[2] if len(ch) > 2 else [],
            "msk": ch[3][0] if len(ch) > 3 else 0}
