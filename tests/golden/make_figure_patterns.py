"""Transcribe the nonzero patterns drawn in the paper's Figures 3, 4 and 5.

The figures show the butterfly factorization of a 64 x 64 complementary
low-rank matrix with L = 6, h = 3, one point per leaf and rank r = 1:
  Fig. 3  the middle-level factorization K ~ U^3 M^3 (V^3)^*;
  Fig. 4  U^3 ~ U^4 G^3 (top) and U^4 ~ U^5 G^4 (bottom);
  Fig. 5  (V^3)^* ~ (H^3)^* (H^4)^* (V^5)^*.
Each grey rectangle in the tikz source is one nonzero entry (0.5 drawing
units per matrix entry, drawing origin at the bottom-left, the top edge at
y = 32 except for M^3 whose top edge is at y = 16).  This script evaluates
the drawing loops of the figures and converts every rectangle into the
(row, column) entries it covers.  It reads nothing but its own constants and
writes `fig_patterns_L6_r1.txt` next to itself.

Run:  python tests/golden/make_figure_patterns.py
"""
import os


def frange(a, b, step):
    out, v = [], a
    while v <= b + 1e-9:
        out.append(v)
        v += step
    return out


def cells(x0, y0, x1, y1, top):
    """Entries covered by the rectangle with corners (x0,y0), (x1,y1)."""
    xa, xb = sorted((x0, x1))
    ya, yb = sorted((y0, y1))
    cols = range(int(round(xa / 0.5)), int(round(xb / 0.5)))
    rows = range(int(round((top - yb) / 0.5)), int(round((top - ya) / 0.5)))
    return {(r, c) for r in rows for c in cols}


def patterns():
    P = {}
    # Fig. 3, second matrix: U^3
    s = set()
    for i in frange(0, 3.5, 0.5):
        for j in frange(0, 28, 4):
            s |= cells(32 - i - j, j, 32 - i - j - 0.5, j + 4, 32)
    P["U3"] = s
    # Fig. 3, third matrix: M^3 (its drawing spans y in [-15.5, 16])
    s = set()
    for i in frange(0, 3.5, 0.5):
        for j in frange(0, 3.5, 0.5):
            s |= cells(8 * i + j, 16 - 8 * j - i, 8 * i + j + 0.5, 15.5 - 8 * j - i, 16)
    P["M3"] = s
    # Fig. 3, fourth matrix: (V^3)^*
    s = set()
    for i in frange(0, 3.5, 0.5):
        for j in frange(0, 28, 4):
            s |= cells(j, 32 - i - j, j + 4, 32 - i - j - 0.5, 32)
    P["V3h"] = s
    # Fig. 4 top, third matrix: U^4
    s = set()
    for k in frange(0, 30, 2):
        for i in frange(0, 1.5, 0.5):
            s |= cells(32 - i - k, k, 32 - i - k - 0.5, k + 2, 32)
    P["U4"] = s
    # Fig. 4 top, fourth matrix: G^3
    s = set()
    for k in frange(0, 28, 4):
        for i in frange(0, 1.5, 0.5):
            s |= cells(32 - 2 * i - k, k + i, 32 - 2 * i - k - 1, k + i + 0.5, 32)
            s |= cells(32 - 2 * i - k, k + i + 2, 32 - 2 * i - k - 1, k + i + 2.5, 32)
    P["G3"] = s
    # Fig. 4 bottom, second matrix: U^5
    s = set()
    for k in frange(0, 31, 1):
        for i in frange(0, 0.5, 0.5):
            s |= cells(32 - i - k, k, 32 - i - k - 0.5, k + 1, 32)
    P["U5"] = s
    # Fig. 4 bottom, third matrix: G^4
    s = set()
    for k in frange(0, 30, 2):
        for i in frange(0, 0.5, 0.5):
            s |= cells(32 - 2 * i - k, k + i, 32 - 2 * i - k - 1, k + i + 0.5, 32)
            s |= cells(32 - 2 * i - k, k + i + 1, 32 - 2 * i - k - 1, k + i + 1.5, 32)
    P["G4"] = s
    # Fig. 5, second matrix: (H^3)^*
    s = set()
    for k in frange(0, 28, 4):
        for i in frange(0, 1.5, 0.5):
            s |= cells(k + i, 32 - 2 * i - k, k + i + 0.5, 32 - 2 * i - k - 1, 32)
            s |= cells(k + i + 2, 32 - 2 * i - k, k + i + 2.5, 32 - 2 * i - k - 1, 32)
    P["H3h"] = s
    # Fig. 5, third matrix: (H^4)^*
    s = set()
    for k in frange(0, 30, 2):
        for i in frange(0, 0.5, 0.5):
            s |= cells(k + i, 32 - 2 * i - k, k + i + 0.5, 32 - 2 * i - k - 1, 32)
            s |= cells(k + i + 1, 32 - 2 * i - k, k + i + 1.5, 32 - 2 * i - k - 1, 32)
    P["H4h"] = s
    # Fig. 5, fourth matrix: (V^5)^*
    s = set()
    for k in frange(0, 31, 1):
        for i in frange(0, 0.5, 0.5):
            s |= cells(k, 32 - i - k, k + 1, 32 - i - k - 0.5, 32)
    P["V5h"] = s
    return P


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    out = os.path.join(here, "fig_patterns_L6_r1.txt")
    with open(out, "w") as fh:
        fh.write("# Nonzero entries of the factors drawn in Figures 3-5 of the paper\n")
        fh.write("# (64 x 64 matrix, L = 6, h = 3, r = 1, one point per leaf).\n")
        fh.write("# Written by make_figure_patterns.py from the figures' tikz loops.\n")
        fh.write("# name row col\n")
        for name, s in patterns().items():
            for (r, c) in sorted(s):
                fh.write(f"{name} {r} {c}\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
