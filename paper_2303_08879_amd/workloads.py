"""Seeded synthetic inputs for the selective Fock-amplitude path.

This module only builds *inputs*: circuit parameters drawn from seeded
generators, the Gaussian moments of the state those circuits prepare, and the
Bargmann triple (A, b, c) that parametrises the state's Fock amplitudes
(Sec. 2.1, Eqs. A_rho / b_rho and the vacuum amplitude rho_0 of Sec. 2.2).
It holds none of the Fock recurrence itself; both the CPU oracle (through the
tests) and the GPU path consume the triples it returns.

Conventions
-----------
* Complex basis xi = (a_1..a_M, a_1^dag..a_M^dag); covariance
  sigma_ij = 1/2 <{dxi_i, dxi_j^dag}>, means mu = <xi>.  Vacuum: sigma = 1/2.
* Fock index order of a density matrix: for each mode a (ket, bra) pair with
  rho_{m,n} = <m|rho|n>, so the ket index carries the state vector psi and the
  bra index its conjugate.
* The triple is returned in *block order* [ket_1..ket_M, bra_1..bra_M].  The
  paper's block formulas put the conjugated (bra) block first: its b for a
  coherent state is [conj(alpha); alpha].  Swapping the two blocks of a
  physical state equals complex conjugation, so the ket-first triple is the
  complex conjugate of the paper's expressions:
      A = conj(P sigma_- sigma_+^{-1}),  b = conj(P sigma_+^{-1} mu),
      c = exp(-1/2 mu^dag sigma_+^{-1} mu) / sqrt(det sigma_+).
  The tests pin this reading against the coherent state and against the
  moments <a>, <a a>, <a^dag a> that sigma and mu define.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "haar_unitary",
    "gaussian_moments",
    "bargmann_triple",
    "Circuit",
    "config1",
    "config2",
    "config3",
    "config4",
    "config5",
    "config5b",
    "pure_state",
    "state8",
    "random_cotangent",
]


def haar_unitary(rng: np.random.Generator, M: int) -> np.ndarray:
    """Haar-random M x M unitary: QR of a complex Ginibre matrix with the phases
    of R's diagonal divided out (Mezzadri's construction).  Draw order: the real
    part, then the imaginary part."""
    re = rng.standard_normal((M, M))
    im = rng.standard_normal((M, M))
    Z = (re + 1j * im) / np.sqrt(2.0)
    Q, R = np.linalg.qr(Z)
    d = np.diag(R)
    return Q * (d / np.abs(d))[None, :]


def gaussian_moments(r, U, eta, alpha=None):
    """Complex-basis covariance sigma (2M x 2M) and means mu (2M) of the state
    prepared by: single-mode squeezers S(r_j) (real r, x-squeezed) on vacuum,
    then displacements alpha_j, then the interferometer U, then pure loss
    eta_j on every mode just before detection."""
    r = np.asarray(r, dtype=np.float64)
    M = r.shape[0]
    U = np.asarray(U, dtype=np.complex128)
    eta = np.broadcast_to(np.asarray(eta, dtype=np.float64), (M,))
    if alpha is None:
        alpha = np.zeros(M, dtype=np.complex128)
    alpha = np.asarray(alpha, dtype=np.complex128)

    ch, sh = np.cosh(r), np.sinh(r)
    # Bogoliubov map of the squeezers on (a, a^dag): a -> cosh r a - sinh r a^dag.
    Ws = np.block([[np.diag(ch), -np.diag(sh)], [-np.diag(sh), np.diag(ch)]]).astype(np.complex128)
    sigma = 0.5 * Ws @ Ws.conj().T
    mu = np.concatenate([alpha, alpha.conj()])
    # Passive interferometer a -> U a, a^dag -> conj(U) a^dag.
    Wu = np.block([[U, np.zeros((M, M))], [np.zeros((M, M)), U.conj()]])
    sigma = Wu @ sigma @ Wu.conj().T
    mu = Wu @ mu
    # Pure loss: a -> sqrt(eta) a + sqrt(1-eta) vacuum.
    s = np.sqrt(np.concatenate([eta, eta]))
    sigma = s[:, None] * sigma * s[None, :] + np.diag(0.5 * (1.0 - s * s))
    mu = s * mu
    return sigma, mu


def bargmann_triple(sigma, mu):
    """(A, b, c) in block order [ket; bra] from the complex covariance and means
    (Sec. 2.1 Eqs. A_rho and b_rho, Sec. 2.2 vacuum amplitude), read ket-first
    as described in the module docstring.  A is returned exactly symmetrised."""
    sigma = np.asarray(sigma, dtype=np.complex128)
    mu = np.asarray(mu, dtype=np.complex128)
    D = sigma.shape[0]
    M = D // 2
    I = np.eye(D)
    sp = sigma + 0.5 * I
    sm = sigma - 0.5 * I
    P = np.block([[np.zeros((M, M)), np.eye(M)], [np.eye(M), np.zeros((M, M))]])
    spinv = np.linalg.inv(sp)
    A = np.conj(P @ sm @ spinv)
    A = 0.5 * (A + A.T)
    b = np.conj(P @ spinv @ mu)
    quad = (mu.conj() @ spinv @ mu).real
    det = np.linalg.det(sp).real
    c = np.exp(-0.5 * quad) / np.sqrt(det)
    return A, b, complex(c)


@dataclass
class Circuit:
    """One workload instance: the triple plus the problem shape.

    ``cutoffs[j]`` is mode j's Fock cutoff; bit j of ``detected_mask`` marks
    mode j as detected (PNR); undetected modes keep their full ket/bra block.
    """

    A: np.ndarray
    b: np.ndarray
    c: complex
    cutoffs: list
    detected_mask: int
    params: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return len(self.cutoffs)

    @property
    def out_shape(self) -> tuple:
        U = [j for j in range(self.M) if not (self.detected_mask >> j) & 1]
        D = [j for j in range(self.M) if (self.detected_mask >> j) & 1]
        return tuple([self.cutoffs[j] for j in U] * 2 + [self.cutoffs[j] for j in D])


def _circuit(rng, M, r_lo, r_hi, eta_fn, cutoffs, detected_mask, alpha_var=0.0, extra=None):
    r = rng.uniform(r_lo, r_hi, size=M)
    U = haar_unitary(rng, M)
    eta = eta_fn(rng, M)
    if alpha_var > 0.0:
        sd = np.sqrt(alpha_var / 2.0)
        alpha = rng.normal(0.0, sd, size=M) + 1j * rng.normal(0.0, sd, size=M)
    else:
        alpha = np.zeros(M, dtype=np.complex128)
    sigma, mu = gaussian_moments(r, U, eta, alpha)
    A, b, c = bargmann_triple(sigma, mu)
    params = dict(r=r, U=U, eta=eta, alpha=alpha, sigma=sigma, mu=mu)
    if extra:
        params.update(extra)
    return Circuit(A, b, c, list(cutoffs), detected_mask, params)


def config1(seed: int = 1) -> Circuit:
    """M=2, both modes detected, cutoff 10; r~U(0.2,0.8), Haar 2x2, eta=0.9, b=0."""
    rng = np.random.default_rng(seed)
    return _circuit(rng, 2, 0.2, 0.8, lambda g, M: np.full(M, 0.9), [10, 10], 0b11)


def config2(seed: int = 2, c_u: int = 30, c_d: int = 12) -> Circuit:
    """M=4; mode 0 undetected (cutoff 30), modes 1..3 detected (cutoff 12);
    r~U(0.3,1.0), Haar 4x4, eta~U(0.85,0.98), displacements alpha~CN(0,0.1)."""
    rng = np.random.default_rng(seed)
    return _circuit(rng, 4, 0.3, 1.0, lambda g, M: g.uniform(0.85, 0.98, size=M),
                    [c_u, c_d, c_d, c_d], 0b1110, alpha_var=0.1)


def config3(seed: int = 3, n: int = 256) -> list:
    """A batch of n independent circuits of uneven shape: M~U{3..6}, each mode's
    cutoff ~U{8..16}, one undetected mode with probability 1/2 (cutoff
    ~U{20..40}, position uniform), r~U(0.1,1.2), Haar, eta~U(0.7,1.0), b=0.
    Shapes are drawn first (one generator), circuit parameters second."""
    rng = np.random.default_rng(seed)
    shapes = []
    for _ in range(n):
        M = int(rng.integers(3, 7))
        cut = [int(x) for x in rng.integers(8, 17, size=M)]
        mask = (1 << M) - 1
        if rng.random() < 0.5:
            u = int(rng.integers(0, M))
            cut[u] = int(rng.integers(20, 41))
            mask &= ~(1 << u)
        shapes.append((M, cut, mask))
    out = []
    for (M, cut, mask) in shapes:
        out.append(_circuit(rng, M, 0.1, 1.2, lambda g, MM: g.uniform(0.7, 1.0, size=MM), cut, mask))
    return out


def config4(seed: int = 4, c_u: int = 40, c_d: int = 10) -> Circuit:
    """M=5; mode 0 undetected (cutoff 40), 4 detected modes (cutoff 10);
    r~U(0.3,1.0), Haar 5x5, eta~U(0.85,0.98), b=0; a seeded normalised target
    psi ~ CN(0,1)^c_u and the conditioning pattern n*=(1,1,1,1)."""
    rng = np.random.default_rng(seed)
    circ = _circuit(rng, 5, 0.3, 1.0, lambda g, M: g.uniform(0.85, 0.98, size=M),
                    [c_u] + [c_d] * 4, 0b11110)
    psi = rng.standard_normal(c_u) + 1j * rng.standard_normal(c_u)
    circ.params["psi_target"] = psi / np.linalg.norm(psi)
    circ.params["n_star"] = (1, 1, 1, 1)
    return circ


def config5(seed: int = 5, c: int = 8) -> Circuit:
    """M=8, all detected, cutoff 8; r~U(0.5,1.0), Haar 8x8, eta~U(0.8,0.95), b=0."""
    rng = np.random.default_rng(seed)
    return _circuit(rng, 8, 0.5, 1.0, lambda g, M: g.uniform(0.8, 0.95, size=M), [c] * 8, 0xFF)


def config5b(seed: int = 55, n: int = 64, c_u: int = 30, c_d: int = 8) -> list:
    """n circuits with M=6: mode 0 undetected (cutoff 30), 5 detected (cutoff 8);
    r~U(0.5,1.0), Haar, eta~U(0.8,0.95), b=0, each with its own target psi for
    the fidelity-type loss at n*=(1,1,1,1,1)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        circ = _circuit(rng, 6, 0.5, 1.0, lambda g, M: g.uniform(0.8, 0.95, size=M),
                        [c_u] + [c_d] * 5, 0b111110)
        psi = rng.standard_normal(c_u) + 1j * rng.standard_normal(c_u)
        circ.params["psi_target"] = psi / np.linalg.norm(psi)
        circ.params["n_star"] = (1, 1, 1, 1, 1)
        out.append(circ)
    return out


def pure_state(seed: int, M: int, cutoffs, r_lo=0.3, r_hi=0.7, alpha_var=0.0) -> Circuit:
    """A lossless circuit (squeezing r~U(r_lo, r_hi), Haar interferometer,
    eta = 1, optional displacement) as a *state-vector* triple: the ket block
    of its density triple, A_psi = A[:M, :M], b_psi = b[:M], and c_psi =
    sqrt(c) (c of a density matrix is |c_psi|^2; the global phase is free).
    For a pure state the ket-bra block of A vanishes (Sec. 2.2, rank-one
    states), which is checked here.  ``detected_mask`` is all modes."""
    rng = np.random.default_rng(seed)
    circ = _circuit(rng, M, r_lo, r_hi, lambda g, MM: np.ones(MM), cutoffs, (1 << M) - 1, alpha_var=alpha_var)
    A, b, c = circ.A, circ.b, circ.c
    assert np.abs(A[:M, M:]).max() < 1e-10, "lossless circuit did not give a pure state"
    circ.params["rho_triple"] = (A, b, c)
    circ.A = np.ascontiguousarray(A[:M, :M])
    circ.b = np.ascontiguousarray(b[:M])
    circ.c = complex(np.sqrt(complex(c)))
    return circ


def state8(seed: int = 8, c: int = 8, alpha_var: float = 0.0) -> Circuit:
    """Pure-state workload: M=8 squeezed modes (r~U(0.3,0.7)) through a Haar
    interferometer, no loss, b=0 (Gaussian boson sampling input), cutoff 8 in
    every mode: psi has 8^8 = 16.8M amplitudes."""
    return pure_state(seed, 8, [c] * 8, alpha_var=alpha_var)


def random_cotangent(shape, seed: int) -> np.ndarray:
    """Seeded dense complex cotangent of a given shape (unit-variance entries)."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)
