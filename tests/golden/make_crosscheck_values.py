"""Writes crosscheck_values.json: states and draws of the paper's example
instance (n = 4294967087, e = 9; skip generator p = 2^31 - 1, a = 784588716;
Sec. II and Figs. 3-4) from the base state (m_0, s_0) = (0, 1), computed
here from algorithm (9) and eq. (7) with plain Python integers.  This script
imports neither the oracle nor the library, so the values pin both.

    python tests/golden/make_crosscheck_values.py
"""

import json
import os

N, E, P, A = 4294967087, 9, 2147483647, 784588716


def main():
    ks = [1, 2, 3, 4, 5, 1000000]
    rows = []
    m, s, usum = 0, 1, 0
    for k in range(1, ks[-1] + 1):
        s = (A * s) % P            # (9a)
        m = (m + s) % N            # (9b)
        usum += s                  # the skip sum of eq. (7b), as an exact integer
        if k in ks:
            c = pow(m, E, N)       # (9c), eq. (1)
            r = (c + 1) / (N + 1)  # (9d): Python's int / int is the correctly rounded quotient
            rows.append({"k": k, "s": s, "m": m, "c": c, "R": r.hex(), "R_repr": repr(r)})
    out = {
        "_comment": "Algorithm (9) from (m_0, s_0) = (0, 1) for the example instance of Sec. II (Figs. 3-4); "
                    "draw k returns c_k (the first draw from position 0 is c_1).  Written by "
                    "tests/golden/make_crosscheck_values.py from plain Python integers.",
        "n": N, "e": E, "p": P, "a": A,
        "draws": rows,
        "U_1e6": usum,
        "full_period_skip_sum_mod_n": (P * (P - 1) // 2) % N,
        "a_inverse_mod_p": pow(A, -1, P),
        "d": pow(E, -1, N - 1),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "crosscheck_values.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(path)


if __name__ == "__main__":
    main()
