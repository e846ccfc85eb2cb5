"""Writes the closed-form fixtures in this folder.

Nothing here runs a kernel or the oracle: every value is a closed form.

* lap2d_N4_quadratic.txt -- y = A x for the 5-point Laplacian on a 4 x 4 grid
  (Dirichlet, diagonal 4, off-diagonal -1) with x(i, j) = i^2 + j^2.  The
  centred second difference is exact on quadratics, so
  y(i, j) = -(p_xx + p_yy) + sum of p over the out-of-grid neighbours
          = -4 + sum_{(a, b) neighbour outside the grid} (a^2 + b^2).
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def lap2d_quadratic(N):
    rows = []
    for i in range(N):
        for j in range(N):
            y = -4
            for a, b in ((i - 1, j), (i + 1, j), (i, j - 1), (i, j + 1)):
                if not (0 <= a < N and 0 <= b < N):
                    y += a * a + b * b
            rows.append((i, j, i * i + j * j, y))
    return rows


def main():
    with open(os.path.join(HERE, "lap2d_N4_quadratic.txt"), "w") as f:
        f.write("# 5-point Laplacian, N=4, Dirichlet, 4/-1; x(i,j)=i^2+j^2; columns: i j x y\n")
        for i, j, x, y in lap2d_quadratic(4):
            f.write(f"{i} {j} {x} {y}\n")


if __name__ == "__main__":
    main()
