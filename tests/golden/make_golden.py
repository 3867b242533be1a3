"""Write the Pascal fixture from the binomial closed form (no oracle, no GPU).

P_ij = C(i+j, i) (symmetric Pascal matrix), L_ij = C(i, j) (lower Pascal
matrix) and P = L L^T (Edelman & Strang, "Pascal Matrices", 2004)."""
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def main(n: int = 8):
    path = os.path.join(HERE, f"pascal{n}_chol.txt")
    with open(path, "w") as f:
        f.write(f"# symmetric Pascal matrix P (n={n}) then its lower Cholesky factor L\n")
        f.write("# P_ij = C(i+j, i); L_ij = C(i, j); P = L L^T "
                "(Edelman & Strang, Amer. Math. Monthly 111, 2004)\n")
        for i in range(n):
            f.write(" ".join(str(math.comb(i + j, i)) for j in range(n)) + "\n")
        f.write("#\n")
        for i in range(n):
            f.write(" ".join(str(math.comb(i, j)) for j in range(n)) + "\n")


if __name__ == "__main__":
    main()
