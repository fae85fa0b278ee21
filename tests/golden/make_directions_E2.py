"""Writes directions_E2.txt: the direction set at direction level E = 2 as
exact integer vectors (Sec. 4.1.2).

Each face of the cube [-1, 1]^3 is split into a 4 x 4 grid of square patches;
a direction is the centre of a patch projected on the unit sphere.  Scaled by
4, a patch centre has the face coordinate +-4 and the two free coordinates
(in increasing axis order) in {-3, -1, 1, 3}, so the direction is the integer
vector n over sqrt(|n|^2), with |n|^2 in {18, 26, 34}.  Index = face * 16 +
i * 4 + j (faces +x, -x, +y, -y, +z, -z; i, j count the patches along the two
free axes); the father at E = 1 is the 2 x 2 patch that contains the patch:
face * 4 + (i // 2) * 2 + (j // 2).

Plain integer enumeration of that construction: it calls neither the oracle
nor the library.
"""
import os

ODD = (-3, -1, 1, 3)


def rows():
    out = []
    for face in range(6):
        axis, sign = face // 2, (1 if face % 2 == 0 else -1)
        free = [a for a in range(3) if a != axis]
        for i, ci in enumerate(ODD):
            for j, cj in enumerate(ODD):
                n = [0, 0, 0]
                n[axis] = 4 * sign
                n[free[0]] = ci
                n[free[1]] = cj
                idx = face * 16 + i * 4 + j
                father = face * 4 + (i // 2) * 2 + (j // 2)
                out.append((idx, *n, sum(c * c for c in n), father))
    return out


if __name__ == "__main__":
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "directions_E2.txt")
    with open(path, "w") as fh:
        fh.write("# Directions at direction level E=2 (Sec. 4.1.2), written by make_directions_E2.py.\n")
        fh.write("# direction = (nx, ny, nz) / sqrt(n2); columns: index nx ny nz n2 father(E=1)\n")
        for r in rows():
            fh.write(" ".join(str(v) for v in r) + "\n")
