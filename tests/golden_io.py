"""Readers for the hand-transcribed figure fixtures under tests/golden/."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line


def read_position_grids(name):
    """{uplo: [[int or None]]} from the Figure 1 / Figure 2 fixtures."""
    out, cur = {}, None
    for line in _lines(name):
        if line.startswith("uplo"):
            cur = line.split()[1]
            out[cur] = []
        else:
            out[cur].append([None if t == "." else int(t) for t in line.split()])
    return out


def read_layout_grids(name):
    """[(transr, uplo, n, [[(i, j, p or None)]])] from the Figure 4 / 6 fixtures
    (i, j, p 1-based)."""
    out = []
    for line in _lines(name):
        if line.startswith("layout"):
            _, t, u, n = line.split()
            out.append((t, u, int(n), []))
        else:
            row = []
            for cell in line.split():
                lab, _, p = cell.partition(":")
                row.append((int(lab[0]), int(lab[1]), int(p) if p else None))
            out[-1][3].append(row)
    return out


def read_printed_positions(name):
    out = []
    for line in _lines(name):
        t, u, n, i, j, p = line.split()
        out.append((t, u, int(n), int(i), int(j), int(p)))
    return out
