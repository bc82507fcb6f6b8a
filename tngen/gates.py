"""Gate matrices (complex128, numpy) for the synthetic circuits.

Conventions (the paper names the gate set but prints no matrices, so these are
the readings used throughout; both the circuit file and every consumer take
the matrices from here, so a phase convention cannot make the two sides
disagree):

* fSim(theta, phi) in the basis |00>,|01>,|10>,|11>:
  [[1,0,0,0],[0,cos t,-i sin t,0],[0,-i sin t,cos t,0],[0,0,0,exp(-i phi)]]
  (Sec. 4, Fig. 6 names fSim as the only two-qubit gate of Sycamore-53).
* sqrt(P) = ((1+i) I + (1-i) P) / 2 for P in {X, Y, W}, W = (X+Y)/sqrt(2).
* Haar unitaries: QR of a complex Ginibre matrix with the phase of R's
  diagonal divided out (Mezzadri, "How to generate random matrices from the
  classical compact groups", 2007).
"""

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
W = (X + Y) / np.sqrt(2.0)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
CNOT = np.array([[1, 0, 0, 0],
                 [0, 1, 0, 0],
                 [0, 0, 0, 1],
                 [0, 0, 1, 0]], dtype=np.complex128)


def sqrt_pauli(p):
    """Principal square root of an involutory Hermitian 2x2 matrix P."""
    return ((1 + 1j) * I2 + (1 - 1j) * p) / 2.0


SQRT_X = sqrt_pauli(X)
SQRT_Y = sqrt_pauli(Y)
SQRT_W = sqrt_pauli(W)
ONE_QUBIT_SET = (SQRT_X, SQRT_Y, SQRT_W)
ONE_QUBIT_NAMES = ("sqrt_x", "sqrt_y", "sqrt_w")


def fsim(theta, phi):
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[1, 0, 0, 0],
                     [0, c, -1j * s, 0],
                     [0, -1j * s, c, 0],
                     [0, 0, 0, np.exp(-1j * phi)]], dtype=np.complex128)


def haar_unitary(d, rng):
    """Haar-random d x d unitary drawn from ``rng`` (numpy Generator)."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[None, :]


# ---------------------------------------------------------------------------
# Optical gates in the Fock basis truncated at cutoff d (photon numbers
# 0 .. d-1), for the GBS circuits of Alg. 1: the squeezer S(r) and the beam
# splitter BS(theta, phi).  The paper names the gates but prints no matrix
# elements; these are the textbook operators,
#   S(z)  = exp((conj(z) a^2 - z adag^2) / 2),          z = r exp(i psi),
#   BS    = exp(theta (exp(i phi) a bdag - exp(-i phi) adag b)),
# and the truncated gate is the block of the exact operator on the kept
# photon numbers (not the exponential of a truncated generator).

def _annihilation(D):
    return np.diag(np.sqrt(np.arange(1, D, dtype=np.float64)), 1).astype(np.complex128)


def squeezer(r, d, psi=0.0, extra=96):
    """<m|S(r e^{i psi})|n> for m, n < d.  S does not conserve photon number,
    so the exact operator's block is computed in a space of d + ``extra``
    photon numbers, where it has converged to rounding for r <= 1."""
    from scipy.linalg import expm
    D = d + extra
    a = _annihilation(D)
    z = r * np.exp(1j * psi)
    gen = 0.5 * (np.conj(z) * (a @ a) - z * (a.T @ a.T))
    return expm(gen)[:d, :d]


def beam_splitter(theta, phi, d):
    """Two-mode BS(theta, phi) truncated at d photons per mode, as the matrix
    U[d*m_a + m_b, d*n_a + n_b] (first mode most significant).  BS conserves
    the total photon number, so on a two-mode space with 2d - 1 photon
    numbers per mode every state of total <= 2d - 2 keeps all of its images:
    the exponential there is exact on the block that is kept."""
    from scipy.linalg import expm
    D = 2 * d - 1
    a1 = _annihilation(D)
    eye = np.eye(D, dtype=np.complex128)
    a = np.kron(a1, eye)        # first mode
    b = np.kron(eye, a1)        # second mode
    gen = theta * (np.exp(1j * phi) * (a @ b.conj().T) - np.exp(-1j * phi) * (a.conj().T @ b))
    U = expm(gen)
    keep = np.array([m * D + n for m in range(d) for n in range(d)])
    return U[np.ix_(keep, keep)]
