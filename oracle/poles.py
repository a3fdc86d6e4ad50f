"""FP64 CPU oracle of the pole search of Eqs.(6)-(10) of arXiv 1501.01752.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg; never by the product library.

The paper's section on mode propagation treats a zeroth-order field
component xi as a meromorphic function of the incident wave-vector modulus
kappa = |k_inc| at fixed frequency and direction (Eq.(6)): simple poles eta_j
(the propagation constants of the modes, n_eff = eta / k0) with amplitudes
zeta_j, plus a regular part.  With P(kappa) = prod_j (kappa - eta_j) =
sum_k p_k kappa^k (Eq.(7), p_Np = 1) the product P xi is analytic, so its
N_d-th Newton divided difference over N_d + 1 points nearly vanishes
(Eq.(8)).  Written out, each point set gives one linear equation in the p_k
(Eq.(9)); N_p point sets give a square system.  The poles are the
eigenvalues of the companion matrix of P, and the amplitudes follow from the
Lagrange interpolant of P xi at the poles (Eq.(10)).

Readings where the printed equations are garbled or silent:
* Eq.(9): xi_i multiplies the weights (it is printed in a denominator).  The
  divided difference of f over kappa_0..kappa_Nd is
  sum_i f(kappa_i) / prod_{j != i}(kappa_i - kappa_j), and f = P xi.
* "N_p - 1 point sets": N_p sets are needed for N_p unknowns p_0..p_{Np-1}.
  The sets are the N_p windows of N_d + 1 consecutive points of one
  equidistant mesh of N_d + N_p points over [kappa_min, kappa_max].
* Eq.(10): the first product runs to N_p (printed "m"); the interpolation
  nodes are those of the middle window (index (N_p - 1) // 2).
"""
import numpy as np


def kappa_mesh(kappa_min, kappa_max, n_poles, n_div):
    """The equidistant mesh of N_d + N_p points (see the readings above)."""
    return np.linspace(float(kappa_min), float(kappa_max), n_div + n_poles)


def divided_difference_weights(kappa):
    """w_i = 1 / prod_{j != i} (kappa_i - kappa_j): the N-th divided difference
    of f over the points is sum_i w_i f(kappa_i)."""
    kappa = np.asarray(kappa, dtype=np.complex128)
    d = kappa[:, None] - kappa[None, :]
    np.fill_diagonal(d, 1.0)
    return 1.0 / np.prod(d, axis=1)


def polynomial_coefficients(kappa, xi, n_poles, n_div):
    """p_0 .. p_{Np-1} of Eq.(9) (p_Np = 1): one equation per window."""
    kappa = np.asarray(kappa, dtype=np.complex128)
    xi = np.asarray(xi, dtype=np.complex128)
    A = np.zeros((n_poles, n_poles), dtype=np.complex128)
    rhs = np.zeros(n_poles, dtype=np.complex128)
    for s in range(n_poles):
        kk = kappa[s:s + n_div + 1]
        wx = divided_difference_weights(kk) * xi[s:s + n_div + 1]
        for k in range(n_poles):
            A[s, k] = np.sum(kk ** k * wx)
        rhs[s] = -np.sum(kk ** n_poles * wx)
    return np.linalg.solve(A, rhs)


def companion_roots(p):
    """Zeros of kappa^Np + sum_{k<Np} p_k kappa^k: eigenvalues of the
    companion matrix (ones on the subdiagonal, -p_k in the last column)."""
    n = len(p)
    C = np.zeros((n, n), dtype=np.complex128)
    C[np.arange(1, n), np.arange(n - 1)] = 1.0
    C[:, -1] = -np.asarray(p, dtype=np.complex128)
    return np.linalg.eigvals(C)


def residues(kappa, xi, eta):
    """Eq.(10): zeta_k = [prod_{i != k} (eta_k - eta_i)]^-1 *
    sum_i xi_i P(kappa_i) prod_{j != i} (eta_k - kappa_j) / (kappa_i - kappa_j),
    over the nodes kappa_0..kappa_Nd given."""
    kappa = np.asarray(kappa, dtype=np.complex128)
    xi = np.asarray(xi, dtype=np.complex128)
    eta = np.asarray(eta, dtype=np.complex128)
    P = np.array([np.prod(kk - eta) for kk in kappa])
    out = np.zeros(len(eta), dtype=np.complex128)
    for k in range(len(eta)):
        lag = np.array([np.prod([(eta[k] - kappa[j]) / (kappa[i] - kappa[j])
                                 for j in range(len(kappa)) if j != i]) for i in range(len(kappa))])
        den = np.prod([eta[k] - eta[i] for i in range(len(eta)) if i != k])
        out[k] = np.sum(xi * P * lag) / den
    return out


def pole_search(kappa, xi, n_poles, n_div):
    """Poles and amplitudes from samples xi_i = xi(kappa_i) on the mesh of
    kappa_mesh: (eta, zeta), eta sorted by real part."""
    p = polynomial_coefficients(kappa, xi, n_poles, n_div)
    eta = companion_roots(p)
    eta = eta[np.argsort(eta.real, kind="stable")]
    mid = (n_poles - 1) // 2
    zeta = residues(np.asarray(kappa)[mid:mid + n_div + 1], np.asarray(xi)[mid:mid + n_div + 1], eta)
    return eta, zeta


def dominant_pole(eta, zeta, kappa_min, kappa_max):
    """The pole of largest |zeta| among those with real part inside
    [kappa_min, kappa_max] and imaginary part at most half the window's
    width (index into eta), or -1 if there is none.  The modes of a lossless
    medium are real poles; poles far off the real axis only model the
    regular part of xi (the paper takes N_p above the two modes of a
    direction for that reason), and under rounding-level changes of the
    samples such a pole can wander into the window with a large amplitude."""
    best, idx = -1.0, -1
    half = 0.5 * (kappa_max - kappa_min)
    for j, (e, z) in enumerate(zip(eta, zeta)):
        if kappa_min <= e.real <= kappa_max and abs(e.imag) <= half and abs(z) > best:
            best, idx = abs(z), j
    return idx
