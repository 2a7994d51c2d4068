"""Reader for tests/golden/small_graphs.txt."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def small_graphs():
    """Yield (name, n, edges, core) from the golden file."""
    with open(os.path.join(HERE, "small_graphs.txt")) as f:
        lines = [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]
    i = 0
    while i < len(lines):
        name = lines[i].split(None, 1)[1]
        n, m = map(int, lines[i + 1].split())
        edges = [tuple(map(int, lines[i + 2 + j].split())) for j in range(m)]
        core = list(map(int, lines[i + 2 + m].split()[1:]))
        yield name, n, edges, core
        i += 3 + m
