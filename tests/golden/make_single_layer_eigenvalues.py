"""Writes single_layer_eigenvalues.txt: closed-form eigenvalues of the KFBI operator A.

For a circle (sphere) of radius R in free space, the single layer with density
cos(m t) (a zonal harmonic Y_l) solves the modified Helmholtz equation inside and
outside with continuous value and flux jump psi (Sec. 5.1, eq. single).  The
interior normal flux is lambda * psi with
    2D: lambda = I_m'(x) K_m(x) / (I_m'(x) K_m(x) - I_m(x) K_m'(x)),  x = sqrt(kappa/sigma) R
    3D: the same with the modified spherical Bessel functions i_l, k_l.
The box boundary changes these by about exp(-2 sqrt(kappa) * 0.7) ~ 1e-12 for the
circle/sphere of radius 0.5 centred in [-1.2, 1.2]^d at kappa = 400.
Only scipy.special is used (no oracle or library code).
"""
import os

from scipy import special


def lam2(m, x):
    return special.ivp(m, x) * special.kv(m, x) / (special.ivp(m, x) * special.kv(m, x) - special.iv(m, x) * special.kvp(m, x))


def lam3(l, x):
    i, k = special.spherical_in(l, x), special.spherical_kn(l, x)
    ip, kp = special.spherical_in(l, x, True), special.spherical_kn(l, x, True)
    return ip * k / (ip * k - i * kp)


if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "single_layer_eigenvalues.txt")
    with open(out, "w") as fh:
        fh.write("# dim mode x=sqrt(kappa/sigma)*R lambda   (kappa=400, sigma=1, R=0.5 -> x=10)\n")
        for m in (0, 1, 5):
            fh.write(f"2 {m} 10.0 {lam2(m, 10.0):.6f}\n")
        for l in (0, 1, 2):
            fh.write(f"3 {l} 10.0 {lam3(l, 10.0):.6f}\n")
