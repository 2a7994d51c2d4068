"""Write tests/golden/small_graphs.txt: small graphs with their oracle coreness.

Calls only the CPU oracle (and the edge-list builders in tests/small_graphs.py).
The file is a regression fixture: the oracle must keep reproducing it, and the
GPU path must match it.  Run:  python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from tests import small_graphs as sg  # noqa: E402

GRAPHS = [
    ("K6", sg.complete(6)),
    ("C9", sg.cycle(9)),
    ("P7", sg.path(7)),
    ("star12", sg.star(12)),
    ("grid5x6", sg.grid(5, 6)),
    ("K3,5", sg.complete_bipartite(3, 5)),
    ("petersen", sg.petersen()),
    ("Q4", sg.hypercube(4)),
    ("wheel7", sg.wheel(7)),
    ("K5+pendant", sg.complete_plus_pendant(5)),
    ("onion", sg.onion([7, 3, 5, 4])),
    ("union", sg.disjoint_union(sg.complete(4), sg.cycle(5), sg.path(3), (2, []))),
    ("random30", sg.random_graph(30, 0.2, 1)),
    ("random40", sg.random_graph(40, 0.35, 2)),
    ("tree25", sg.random_tree(25, 3)),
    ("empty1", (1, [])),
]


def main():
    out = os.path.join(HERE, "small_graphs.txt")
    with open(out, "w") as f:
        f.write("# graph name / n m / m edge lines / coreness line; values from oracle.coreness\n")
        for name, (n, edges) in GRAPHS:
            rp, ci = sg.to_csr(n, edges)
            core = oracle.coreness(rp, ci)
            und = sorted({(min(u, v), max(u, v)) for u, v in edges if u != v})
            f.write(f"graph {name}\n{n} {len(und)}\n")
            for u, v in und:
                f.write(f"{u} {v}\n")
            f.write("core " + " ".join(str(int(c)) for c in core) + "\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
