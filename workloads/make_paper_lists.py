"""Write paper_lists.txt: the fixed number lists behind the array workloads
of the paper's array-performance table (section 8.2) that need primality to
define them.  Every primality decision and factorisation here comes from the
oracle only.  Run from the repository root:

    python -m workloads.make_paper_lists

Sections of the file (one "# name" line, then the numbers, ten a line):

* ``primes_below_2_17``  every prime below 2^17 (the pool that the int16
  primes and the normally distributed primes around 2^16 are drawn from).
* ``largest_prime_below_2_52``  the largest 52-bit prime.
* ``largest_64bit_primes``  the 100 largest primes below 2^64, descending.
* ``largest_composites_factors_gt_2e7``  the 100 largest composites below
  2^64 whose prime factors all exceed 2*10^7, descending (the reading taken
  of the table's "pseudoprimes > 2^53 with factors > 20M").
"""
import os

import numpy as np

import oracle

U64 = (1 << 64) - 1
FACTOR_BOUND = 20_000_000


def prime_factors(n: int) -> list:
    """All prime factors of n (with multiplicity), by the oracle's
    Pollard-Brent search and its primality test."""
    out, stack = [], [n]
    while stack:
        c = stack.pop()
        if c == 1:
            continue
        if oracle.is_prime(c):
            out.append(c)
            continue
        f = oracle.find_factor(c)
        if f in (0, 1, c):
            raise RuntimeError("no factor found for %d" % c)
        stack += [f, c // f]
    return sorted(out)


def main() -> None:
    bits = oracle.sieve_odd(1 << 17)
    idx = np.nonzero(np.unpackbits(bits.view(np.uint8), bitorder="little"))[0]
    small = [2] + [int(2 * i + 1) for i in idx if 2 * i + 1 < (1 << 17)]

    n = (1 << 52) - 1
    while not oracle.is_prime(n):
        n -= 2
    largest52 = n

    primes64, n = [], U64
    while len(primes64) < 100:
        if oracle.is_prime(n):
            primes64.append(n)
        n -= 2

    comps, n = [], U64
    while len(comps) < 100:
        if not oracle.is_prime(n) and min(prime_factors(n)) > FACTOR_BOUND:
            comps.append(n)
        n -= 2

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_lists.txt")
    with open(path, "w") as f:
        f.write("# written by workloads/make_paper_lists.py (oracle primality and factoring)\n")
        for name, vals in (("primes_below_2_17", small),
                           ("largest_prime_below_2_52", [largest52]),
                           ("largest_64bit_primes", primes64),
                           ("largest_composites_factors_gt_2e7", comps)):
            f.write("# %s %d\n" % (name, len(vals)))
            for i in range(0, len(vals), 10):
                f.write(" ".join(str(v) for v in vals[i:i + 10]) + "\n")
    print(len(small), largest52, primes64[:2], comps[:2], comps[-1])


if __name__ == "__main__":
    main()
