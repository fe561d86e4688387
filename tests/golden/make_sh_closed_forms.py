"""Write sh_closed_forms.txt: textbook real-SH closed forms at fixed directions.

The closed forms are the standard table of real spherical harmonics up to
degree 3 (Condon-Shortley phase, z polar axis, index l*l + m + l), e.g. as
derived in any text from Y_lm = N_lm P_l^m(cos theta) e^{i m phi}.  This
script evaluates that table with plain math; it calls neither the oracle nor
the GPU library.  The oracle derives its SH from the general definition
(Legendre recurrence), so the two are independent.
"""
import math
import os

PI = math.pi
TABLE = [
    lambda x, y, z: 1 / (2 * math.sqrt(PI)),
    lambda x, y, z: -math.sqrt(3 / (4 * PI)) * y,
    lambda x, y, z: math.sqrt(3 / (4 * PI)) * z,
    lambda x, y, z: -math.sqrt(3 / (4 * PI)) * x,
    lambda x, y, z: math.sqrt(15 / (4 * PI)) * x * y,
    lambda x, y, z: -math.sqrt(15 / (4 * PI)) * y * z,
    lambda x, y, z: math.sqrt(5 / (16 * PI)) * (3 * z * z - 1),
    lambda x, y, z: -math.sqrt(15 / (4 * PI)) * x * z,
    lambda x, y, z: math.sqrt(15 / (16 * PI)) * (x * x - y * y),
    lambda x, y, z: -math.sqrt(35 / (32 * PI)) * y * (3 * x * x - y * y),
    lambda x, y, z: math.sqrt(105 / (4 * PI)) * x * y * z,
    lambda x, y, z: -math.sqrt(21 / (32 * PI)) * y * (5 * z * z - 1),
    lambda x, y, z: math.sqrt(7 / (16 * PI)) * z * (5 * z * z - 3),
    lambda x, y, z: -math.sqrt(21 / (32 * PI)) * x * (5 * z * z - 1),
    lambda x, y, z: math.sqrt(105 / (16 * PI)) * z * (x * x - y * y),
    lambda x, y, z: -math.sqrt(35 / (32 * PI)) * x * (x * x - 3 * y * y),
]
# unit directions with rational coordinates (Pythagorean quadruples) plus axes
DIRS = [(2, -3, 6, 7), (1, 2, 2, 3), (-4, 4, -7, 9), (0, 0, 1, 1), (1, 0, 0, 1), (0, -1, 0, 1), (6, 2, -3, 7)]


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sh_closed_forms.txt")
    with open(out, "w") as f:
        f.write("# Real SH closed forms (degree <= 3), written by make_sh_closed_forms.py.\n")
        f.write("# columns: x y z (unit vector) followed by Y_0 .. Y_15\n")
        for a, b, c, n in DIRS:
            x, y, z = a / n, b / n, c / n
            vals = [fn(x, y, z) for fn in TABLE]
            f.write(" ".join(repr(v) for v in (x, y, z, *vals)) + "\n")


if __name__ == "__main__":
    main()
