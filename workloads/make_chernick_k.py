"""Write chernick_k.txt: every k >= 1 with (6k+1), (12k+1), (18k+1) prime and
(6k+1)(12k+1)(18k+1) < 2^64.  Primality comes from the oracle's trial
division (O1) only.  Run from the repository root:

    python -m workloads.make_chernick_k
"""
import os

import oracle


def main() -> None:
    ks = []
    k = 1
    while (6 * k + 1) * (12 * k + 1) * (18 * k + 1) < (1 << 64):
        if all(oracle.trial_is_prime(f) for f in (6 * k + 1, 12 * k + 1, 18 * k + 1)):
            ks.append(k)
        k += 1
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "chernick_k.txt")
    with open(path, "w") as f:
        f.write("# k with 6k+1, 12k+1, 18k+1 prime and product < 2^64; "
                "written by workloads/make_chernick_k.py (oracle trial division)\n")
        for i in range(0, len(ks), 10):
            f.write(" ".join(str(x) for x in ks[i:i + 10]) + "\n")
    print(len(ks), ks[:8], ks[-1])


if __name__ == "__main__":
    main()
