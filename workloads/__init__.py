"""Seeded synthetic workloads for the QCL trajectory ensemble.

This module only *defines inputs*: model parameters of linear-vibronic
harmonic (LVC) Hamiltonians, initial-state descriptors and run shapes.  It
contains none of the method's arithmetic (no sampling, no eigen-solves, no
propagation), and it is shared by the FP64 oracle, the HIP path, the tests
and the benchmark, which all consume the *numbers* it produces.

Model family (Sec. II.A, Eq. 1 symbols R, P, M; Sec. II.C models):

    H = sum_j p_j^2/(2 m_j) + sum_j m_j w_j^2 q_j^2 / 2 + V(q),
    V(q) = V0 + sum_j q_j K_j           (V0, K_j real symmetric N x N)

optionally with separable higher powers of each mode (``poly``):

    V(q) += sum_j sum_{k=2..D} q_j^k A_jk   (A_jk real symmetric, D <= 4)

which adds state-dependent frequencies (k = 2) and anharmonicity (k = 3, 4).

Workloads (sizes from the headline configurations; parameters of the
paper's 3-D spin-boson model live in its cited references and are replaced
by an Ohmic discretisation here; the pyrazine-like model uses the
vibronic parameters stated for the conical-intersection workload):

* ``spin_boson_1mode``  1 mode, 2 states, reduced units.
* ``spin_boson_ohmic``  3 modes discretising an Ohmic density, 2 states.
* ``pyrazine_ci``       2-state 3-mode conical-intersection model (eV, fs).
* ``random_lvc``        N-state harmonic models drawn from a seed (batched
                        and served workloads).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

HBAR_EV_FS = 0.6582119569  # hbar in eV*fs (CODATA 2018)

INIT_DIABATIC = 0
INIT_ADIABATIC = 1


@dataclasses.dataclass
class LVCModel:
    """Numbers of one LVC model.  Arrays are float64, C-contiguous."""

    name: str
    mass: np.ndarray   # [M]
    omega: np.ndarray  # [M]
    v0: np.ndarray     # [N, N] symmetric
    k: np.ndarray      # [M, N, N] each symmetric
    hbar: float = 1.0
    time_unit_fs: Optional[float] = None  # fs per internal time unit (eV models)
    poly: Optional[np.ndarray] = None  # [M, D-1, N, N]: A_jk for k = 2..D (D <= 4), each symmetric
    # cross-mode bilinear terms q_i q_j B (i != j), B [N, N] symmetric
    bilinear: Optional[List[Tuple[int, int, np.ndarray]]] = None

    def __post_init__(self):
        self.mass = np.ascontiguousarray(self.mass, dtype=np.float64)
        self.omega = np.ascontiguousarray(self.omega, dtype=np.float64)
        self.v0 = np.ascontiguousarray(self.v0, dtype=np.float64)
        self.k = np.ascontiguousarray(self.k, dtype=np.float64)
        if self.poly is not None:
            self.poly = np.ascontiguousarray(self.poly, dtype=np.float64)
        if self.bilinear is not None:
            self.bilinear = [(int(i), int(j), np.ascontiguousarray(B, dtype=np.float64)) for i, j, B in self.bilinear]

    @property
    def degree(self) -> int:
        """Highest power of q_j in V(q): 1 for an LVC model."""
        return 1 if self.poly is None else int(self.poly.shape[1]) + 1

    @property
    def n_states(self) -> int:
        return int(self.v0.shape[0])

    @property
    def n_modes(self) -> int:
        return int(self.mass.shape[0])


@dataclasses.dataclass
class SourceModel:
    """A model whose diabatic potential matrix V(q) is given as code:
    H = sum_j p_j^2 / (2 m_j) + V(q), V holding every q-dependent term.
    ``hip_source`` defines the three device functions of
    qcl_create_model_source (V's upper triangle, the force contraction and
    the velocity coupling); ``c_source`` is a plain C transcription of the
    same formulas for the oracle (``qcl_oracle_potential(q, prm, V)`` with V
    the full N x N matrix, ``qcl_oracle_gradient(j, q, prm, G)`` with
    G = dV/dq_j).  ``omega`` are the frequencies of the harmonic reference
    the Wigner initial state is drawn from."""

    name: str
    n_states_: int
    mass: np.ndarray    # [M]
    omega: np.ndarray   # [M]
    params: np.ndarray  # [P]
    hip_source: str
    c_source: str
    hbar: float = 1.0
    time_unit_fs: Optional[float] = None
    poly = None
    bilinear = None

    def __post_init__(self):
        self.mass = np.ascontiguousarray(self.mass, dtype=np.float64)
        self.omega = np.ascontiguousarray(self.omega, dtype=np.float64)
        self.params = np.ascontiguousarray(self.params, dtype=np.float64)

    @property
    def degree(self) -> int:
        return 1

    @property
    def n_states(self) -> int:
        return int(self.n_states_)

    @property
    def n_modes(self) -> int:
        return int(self.mass.shape[0])

    @property
    def v0(self) -> np.ndarray:  # not used by either path; the shape carries N
        return np.zeros((self.n_states, self.n_states))

    @property
    def k(self) -> np.ndarray:
        return np.zeros((self.n_modes, self.n_states, self.n_states))


@dataclasses.dataclass
class InitSpec:
    """Initial state: thermal Wigner (q, p) centred on q0, electronic state
    ``state`` in the diabatic (default) or adiabatic basis."""

    kT: float
    q0: np.ndarray
    state: int = 0
    basis: int = INIT_DIABATIC

    def __post_init__(self):
        self.q0 = np.ascontiguousarray(self.q0, dtype=np.float64)


@dataclasses.dataclass
class RunSpec:
    n_traj: int
    n_steps: int
    dt: float
    cadence: int
    seed: int

    @property
    def n_out(self) -> int:
        return self.n_steps // self.cadence + 1


@dataclasses.dataclass
class Workload:
    model: LVCModel
    init: InitSpec
    run: RunSpec


def _z_diag(n: int) -> np.ndarray:
    """Per-state bath coupling pattern diag(z_k), z_k = 1 - 2k/(N-1):
    (1,-1) for N=2, (1,0,-1) for N=3, (1,1/3,-1/3,-1) for N=4."""
    return np.diag([1.0 - 2.0 * kk / (n - 1) for kk in range(n)])


def ohmic_modes(n_modes: int, omega_c: float = 1.0, xi: float = 0.1):
    """Discretised Ohmic density J(w) = (pi/2) xi w exp(-w/w_c):
    w_j = -w_c ln(1 - j/(M+1)), c_j = w_j sqrt(xi w_c/(M+1)), j = 1..M."""
    j = np.arange(1, n_modes + 1, dtype=np.float64)
    w = -omega_c * np.log(1.0 - j / (n_modes + 1))
    c = w * math.sqrt(xi * omega_c / (n_modes + 1))
    return w, c


def state1_minimum(model: LVCModel) -> np.ndarray:
    """Minimum of the first diabatic surface: q0_j = -(K_j)_00/(m_j w_j^2)."""
    return -model.k[:, 0, 0] / (model.mass * model.omega ** 2)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def spin_boson_1mode(n_traj: int = 10_000, n_steps: int = 200, dt: float = 0.05,
                     cadence: int = 10, seed: int = 0) -> Workload:
    eps, delta, g = 0.5, 0.2, 0.5
    model = LVCModel(
        name="spin_boson_1mode",
        mass=[1.0], omega=[1.0],
        v0=[[eps, delta], [delta, -eps]],
        k=[[[g, 0.0], [0.0, -g]]],
    )
    init = InitSpec(kT=0.5, q0=state1_minimum(model), state=0)
    return Workload(model, init, RunSpec(n_traj, n_steps, dt, cadence, seed))


def spin_boson_ohmic(kT: float = 0.2, n_traj: int = 1_000_000, n_steps: int = 2000,
                     dt: float = 0.02, cadence: int = 10, seed: Optional[int] = None,
                     n_modes: int = 3) -> Workload:
    w, c = ohmic_modes(n_modes, 1.0, 0.1)
    eps, delta = 0.0, 0.5
    k = np.stack([cj * _z_diag(2) for cj in c])
    model = LVCModel(
        name=f"spin_boson_ohmic_m{n_modes}",
        mass=np.ones(n_modes), omega=w,
        v0=[[eps, delta], [delta, -eps]], k=k,
    )
    init = InitSpec(kT=kT, q0=state1_minimum(model), state=0)
    if seed is None:
        seed = 1 if kT <= 0.5 else 2
    return Workload(model, init, RunSpec(n_traj, n_steps, dt, cadence, seed))


def pyrazine_ci(n_traj: int = 10_000_000, n_steps: int = 1000, dt_fs: float = 0.5,
                cadence: int = 10, seed: int = 3) -> Workload:
    """Two-state three-mode S2/S1 conical-intersection model in dimensionless
    normal coordinates (m_j = 1/w_j so that H_j = w_j (p^2 + q^2)/2), energies
    in eV, hbar = 1 internally, one time unit = hbar/eV = 0.6582 fs."""
    om = np.array([0.126, 0.074, 0.118])  # nu1, nu6a (tuning), nu10a (coupling)
    k = np.zeros((3, 2, 2))
    k[0] = np.diag([0.037, -0.254])
    k[1] = np.diag([-0.105, 0.149])
    k[2] = [[0.0, 0.262], [0.262, 0.0]]
    model = LVCModel(
        name="pyrazine_ci", mass=1.0 / om, omega=om,
        v0=np.diag([-0.46, 0.46]), k=k, hbar=1.0, time_unit_fs=HBAR_EV_FS,
    )
    init = InitSpec(kT=0.0, q0=np.zeros(3), state=1)  # vertical excitation, upper diabatic state
    return Workload(model, init, RunSpec(n_traj, n_steps, dt_fs / HBAR_EV_FS, cadence, seed))


def zero_coupling(n_traj: int = 2000, n_steps: int = 200, dt: float = 0.05,
                  cadence: int = 10, seed: int = 11) -> Workload:
    """Diagonal V(q) with well-separated surfaces: no nonadiabatic coupling."""
    model = LVCModel(
        name="zero_coupling", mass=[1.0, 2.0], omega=[1.0, 0.7],
        v0=np.diag([-1.0, 1.0]),
        k=[np.diag([0.2, -0.1]), np.diag([-0.15, 0.05])],
    )
    init = InitSpec(kT=0.3, q0=np.zeros(2), state=0)
    return Workload(model, init, RunSpec(n_traj, n_steps, dt, cadence, seed))


def uncoupled_harmonic(n_traj: int = 1000, n_steps: int = 300, dt: float = 0.05,
                       cadence: int = 10, seed: int = 12) -> Workload:
    """K_j = 0: every surface is the bare harmonic well."""
    model = LVCModel(
        name="uncoupled_harmonic", mass=[1.0, 0.5, 3.0], omega=[1.0, 1.7, 0.4],
        v0=[[0.3, 0.1], [0.1, -0.3]], k=np.zeros((3, 2, 2)),
    )
    init = InitSpec(kT=0.8, q0=np.array([0.5, -0.2, 1.0]), state=0)
    return Workload(model, init, RunSpec(n_traj, n_steps, dt, cadence, seed))


def random_lvc(index: int, key: int = 4, n_modes: Optional[int] = None,
               n_states: Optional[int] = None, n_traj: Optional[int] = None,
               n_steps: Optional[int] = None, max_modes: int = 64,
               traj_range=(1e4, 1e6), steps_range=(500, 4000),
               dt: float = 0.05, cadence: int = 50) -> Workload:
    """One N-state harmonic model drawn from (key, index): modes U{1..max},
    states U{2..4}, diabatic biases and couplings U[0, 0.5], kT log-U[0.1, 2],
    trajectories log-U over ``traj_range``, steps U over ``steps_range``.
    K_j = c_j diag(z_k) with the Ohmic c_j (xi = 0.1, w_c = 1)."""
    rng = np.random.Generator(np.random.Philox(key=[key, index]))
    M = int(rng.integers(1, max_modes + 1)) if n_modes is None else int(n_modes)
    N = int(rng.integers(2, 5)) if n_states is None else int(n_states)
    bias = rng.uniform(0.0, 0.5, size=N)
    coup = rng.uniform(0.0, 0.5, size=(N, N))
    kT = float(math.exp(rng.uniform(math.log(0.1), math.log(2.0))))
    T = int(round(math.exp(rng.uniform(math.log(traj_range[0]), math.log(traj_range[1]))))) \
        if n_traj is None else int(n_traj)
    S = int(rng.integers(steps_range[0], steps_range[1] + 1)) if n_steps is None else int(n_steps)
    S = max(cadence, (S // cadence) * cadence)
    v0 = np.triu(coup, 1)
    v0 = v0 + v0.T + np.diag(bias - bias.mean())
    w, c = ohmic_modes(M, 1.0, 0.1)
    k = np.stack([cj * _z_diag(N) for cj in c])
    model = LVCModel(name=f"random_lvc_{key}_{index}", mass=np.ones(M), omega=w, v0=v0, k=k)
    init = InitSpec(kT=kT, q0=state1_minimum(model), state=0)
    seed = (key << 32) | (index & 0xFFFFFFFF)
    return Workload(model, init, RunSpec(T, S, dt, cadence, seed))


def pyrazine_qvc(n_traj: int = 1_000_000, n_steps: int = 200, dt_fs: float = 0.5,
                 cadence: int = 2, seed: int = 7) -> Workload:
    """The pyrazine-like model with state-dependent frequencies and a
    quartic tuning mode: V(q) gains sum_j (gamma_j/2) q_j^2 diag(-1, +1) on
    the two totally symmetric modes (the upper state softer along nu6a,
    stiffer along nu1) and (lambda/24) q^4 I on nu6a (energies in eV,
    dimensionless coordinates, as ``pyrazine_ci``)."""
    base = pyrazine_ci(n_traj=n_traj, n_steps=n_steps, dt_fs=dt_fs, cadence=cadence, seed=seed)
    m = base.model
    poly = np.zeros((3, 3, 2, 2))  # powers 2, 3, 4
    poly[0, 0] = 0.5 * 0.012 * np.diag([-1.0, 1.0])   # nu1: gamma = 0.012 eV
    poly[1, 0] = 0.5 * -0.018 * np.diag([-1.0, 1.0])  # nu6a: gamma = -0.018 eV
    poly[1, 2] = (0.004 / 24.0) * np.eye(2)           # nu6a: lambda = 0.004 eV
    model = LVCModel(name="pyrazine_qvc", mass=m.mass, omega=m.omega, v0=m.v0, k=m.k, hbar=m.hbar,
                     time_unit_fs=m.time_unit_fs, poly=poly)
    return Workload(model, base.init, base.run)


def random_poly(index: int, n_states: int = 3, n_modes: int = 5, degree: int = 4, key: int = 6,
                n_traj: int = 2000, n_steps: int = 100, dt: float = 0.05, cadence: int = 10,
                rank_full: bool = True) -> Workload:
    """An N-state model with every power up to ``degree`` in every mode,
    drawn from (key, index).  Linear and higher couplings are dense random
    symmetric matrices (so the coupling space has full rank when
    ``rank_full``), cubic terms are small, and each quartic term is a
    positive multiple of the identity plus a smaller symmetric part, so every
    adiabatic surface is confining."""
    rng = np.random.Generator(np.random.Philox(key=[key, index]))
    N, M = int(n_states), int(n_modes)

    def sym(scale):
        a = rng.uniform(-scale, scale, size=(N, N))
        return 0.5 * (a + a.T)

    bias = np.linspace(-0.4, 0.4, N)
    v0 = np.diag(bias) + sym(0.1) * (1.0 - np.eye(N))
    omega = rng.uniform(0.5, 1.5, size=M)
    mass = rng.uniform(0.7, 1.4, size=M)
    k = np.stack([sym(0.15) if rank_full else 0.15 * rng.uniform(-1, 1) * _z_diag(N) for _ in range(M)])
    poly = np.zeros((M, degree - 1, N, N))
    for j in range(M):
        poly[j, 0] = sym(0.05 * mass[j] * omega[j] ** 2)
        if degree >= 3:
            poly[j, 1] = sym(0.02)
        if degree >= 4:
            poly[j, 2] = 0.05 * np.eye(N) + sym(0.01)
    model = LVCModel(name=f"random_poly_{key}_{index}", mass=mass, omega=omega, v0=v0, k=k, poly=poly)
    init = InitSpec(kT=0.3, q0=np.zeros(M), state=N - 1)
    seed = (key << 32) | (index & 0xFFFFFFFF)
    return Workload(model, init, RunSpec(n_traj, n_steps, dt, cadence, seed))


def pyrazine_bilinear(n_traj: int = 1_000_000, n_steps: int = 200, dt_fs: float = 0.5,
                      cadence: int = 2, seed: int = 9) -> Workload:
    """``pyrazine_qvc`` with two cross-mode bilinear terms: a state-dependent
    mixing of the tuning modes nu1 and nu6a, q_1 q_6a diag(-0.006, 0.008),
    and a bilinear part of the interstate coupling, q_6a q_10a (0.012 sigma_x)
    (eV, dimensionless coordinates)."""
    base = pyrazine_qvc(n_traj=n_traj, n_steps=n_steps, dt_fs=dt_fs, cadence=cadence, seed=seed)
    m = base.model
    bil = [(0, 1, np.diag([-0.006, 0.008])), (1, 2, np.array([[0.0, 0.012], [0.012, 0.0]]))]
    model = LVCModel(name="pyrazine_bilinear", mass=m.mass, omega=m.omega, v0=m.v0, k=m.k, hbar=m.hbar,
                     time_unit_fs=m.time_unit_fs, poly=m.poly, bilinear=bil)
    return Workload(model, base.init, base.run)


def random_bilinear(index: int, n_states: int = 3, n_modes: int = 5, n_pairs: int = 3, degree: int = 2,
                    key: int = 8, n_traj: int = 2000, n_steps: int = 100, dt: float = 0.05,
                    cadence: int = 10, all_pairs: bool = False, shared: bool = False) -> Workload:
    """``random_poly`` with ``n_pairs`` cross-mode bilinear terms on distinct
    random mode pairs (every pair with ``all_pairs``), each coupling a dense
    random symmetric matrix small against the harmonic force constants (the
    surfaces stay confining); with ``shared`` each coupling is a multiple of
    the identity (mode mixing common to all states)."""
    wl = random_poly(index, n_states=n_states, n_modes=n_modes, degree=degree, key=key, n_traj=n_traj,
                     n_steps=n_steps, dt=dt, cadence=cadence)
    rng = np.random.Generator(np.random.Philox(key=[key + 1000, index]))
    N, M = int(n_states), int(n_modes)
    pairs = set()
    if all_pairs:
        pairs = {(i, j) for i in range(M) for j in range(i + 1, M)}
    while len(pairs) < n_pairs:
        i, j = sorted(int(x) for x in rng.choice(M, size=2, replace=False))
        pairs.add((i, j))
    bil = []
    scale = 0.04 / max(1.0, math.sqrt(len(pairs) / 4.0))
    for i, j in sorted(pairs):
        if shared:
            bil.append((i, j, rng.uniform(-scale, scale) * np.eye(N)))
        else:
            a = rng.uniform(-scale, scale, size=(N, N))
            bil.append((i, j, 0.5 * (a + a.T)))
    m = wl.model
    wl.model = LVCModel(name=f"random_bilinear_{key}_{index}", mass=m.mass, omega=m.omega, v0=m.v0, k=m.k,
                        poly=m.poly, bilinear=bil)
    return wl


# Two Morse curves along mode 0 (depth D_s, range a, minima x_s, offset of
# state 1), a harmonic mode 1 shared by both states and shifted linearly on
# state 1, and a diabatic coupling c (c0 + a Gaussian in mode 0 centred
# between the minima) (1 + gamma q_1^2): not separable in the modes, and
# never zero, so the surfaces only come close at an avoided crossing.
# Parameters: D0, D1, a, x0, x1, offset, k1, kappa, c, beta, xc, gamma, c0.
_MORSE_HIP = """
// binary64 and binary32 (templates): the binary32 kernels are built too
#define QCL_SOURCE_FP32 1
template <typename T>
__device__ inline T morse_prm(int i) { return (T)qcl_param[i]; }
template <typename T>
__device__ inline void morse_parts(const T *q, T &e0, T &e1, T &g)
{
    e0 = exp(-morse_prm<T>(2) * (q[0] - morse_prm<T>(3)));
    e1 = exp(-morse_prm<T>(2) * (q[0] - morse_prm<T>(4)));
    const T d = q[0] - morse_prm<T>(10);
    g = exp(-morse_prm<T>(9) * d * d);  // the Gaussian; the coupling's shape is c0 + g
}
template <typename T>
__device__ void qcl_potential(const T *q, T *V)
{
    T e0, e1, g;
    morse_parts(q, e0, e1, g);
    const T h = T(0.5) * morse_prm<T>(6) * q[1] * q[1];
    V[0] = morse_prm<T>(0) * (T(1) - e0) * (T(1) - e0) + h;
    V[1] = morse_prm<T>(8) * (morse_prm<T>(12) + g) * (T(1) + morse_prm<T>(11) * q[1] * q[1]);
    V[2] = morse_prm<T>(1) * (T(1) - e1) * (T(1) - e1) + morse_prm<T>(5) + h + morse_prm<T>(7) * q[1];
}
template <typename T>
__device__ inline void morse_gradient(const T *q, T (&G)[2][3])
{
    T e0, e1, g;
    morse_parts(q, e0, e1, g);
    const T a = morse_prm<T>(2);
    G[0][0] = T(2) * morse_prm<T>(0) * a * e0 * (T(1) - e0);
    G[0][1] = T(-2) * morse_prm<T>(9) * (q[0] - morse_prm<T>(10)) * morse_prm<T>(8) * g *
              (T(1) + morse_prm<T>(11) * q[1] * q[1]);
    G[0][2] = T(2) * morse_prm<T>(1) * a * e1 * (T(1) - e1);
    G[1][0] = morse_prm<T>(6) * q[1];
    G[1][1] = morse_prm<T>(8) * (morse_prm<T>(12) + g) * T(2) * morse_prm<T>(11) * q[1];
    G[1][2] = morse_prm<T>(6) * q[1] + morse_prm<T>(7);
}
template <typename T>
__device__ void qcl_force(const T *q, const T *w, T *f)
{
    T G[2][3];
    morse_gradient(q, G);
    for (int j = 0; j < 2; ++j)
        f[j] = -(w[0] * G[j][0] + w[1] * G[j][1] + w[2] * G[j][2]);
}
template <typename T>
__device__ void qcl_coupling(const T *q, const T *v, T *K)
{
    T G[2][3];
    morse_gradient(q, G);
    for (int s = 0; s < 3; ++s)
        K[s] = v[0] * G[0][s] + v[1] * G[1][s];
}
"""

_MORSE_C = """
void qcl_oracle_potential(const double *q, const double *prm, double *V)
{
    double D0 = prm[0], D1 = prm[1], a = prm[2], x0 = prm[3], x1 = prm[4], off = prm[5];
    double k1 = prm[6], kap = prm[7], c = prm[8], beta = prm[9], xc = prm[10], gam = prm[11], c0 = prm[12];
    double m0 = 1.0 - exp(-a * (q[0] - x0)), m1 = 1.0 - exp(-a * (q[0] - x1));
    double bath = 0.5 * k1 * q[1] * q[1];
    double cpl = c * (c0 + exp(-beta * (q[0] - xc) * (q[0] - xc))) * (1.0 + gam * q[1] * q[1]);
    V[0] = D0 * m0 * m0 + bath;
    V[1] = cpl;
    V[2] = cpl;
    V[3] = D1 * m1 * m1 + off + bath + kap * q[1];
}

void qcl_oracle_gradient(int j, const double *q, const double *prm, double *G)
{
    double D0 = prm[0], D1 = prm[1], a = prm[2], x0 = prm[3], x1 = prm[4];
    double k1 = prm[6], kap = prm[7], c = prm[8], beta = prm[9], xc = prm[10], gam = prm[11], c0 = prm[12];
    double g = c * exp(-beta * (q[0] - xc) * (q[0] - xc));
    if (j == 0) {
        double t0 = exp(-a * (q[0] - x0)), t1 = exp(-a * (q[0] - x1));
        G[0] = 2.0 * D0 * a * t0 * (1.0 - t0);
        G[3] = 2.0 * D1 * a * t1 * (1.0 - t1);
        G[1] = G[2] = -2.0 * beta * (q[0] - xc) * g * (1.0 + gam * q[1] * q[1]);
    } else {
        G[0] = k1 * q[1];
        G[3] = k1 * q[1] + kap;
        G[1] = G[2] = 2.0 * (c * c0 + g) * gam * q[1];
    }
}
"""


def morse_coupled(n_traj: int = 4096, n_steps: int = 200, dt: float = 0.05, cadence: int = 10,
                  seed: int = 11, kT: float = 0.0) -> Workload:
    """Two coupled Morse states with a harmonic spectator mode (reduced
    units, m = 1; each Morse well's harmonic frequency a sqrt(2 D / m) = 1,
    its depth well above the walkers' energy): the walkers start in diabatic
    state 1 at the state-0 minimum and cross the coupling region between the
    minima."""
    params = [5.0, 5.0, 1.0 / math.sqrt(10.0), 0.0, 1.0, 0.2, 1.0, 0.2, 0.15, 1.0, 0.5, 0.3, 0.2]
    model = SourceModel(name="morse_coupled", n_states_=2, mass=[1.0, 1.0], omega=[1.0, 1.0], params=params,
                        hip_source=_MORSE_HIP, c_source=_MORSE_C)
    init = InitSpec(kT=kT, q0=[0.0, 0.0], state=1)
    return Workload(model, init, RunSpec(n_traj, n_steps, dt, cadence, seed))


def lvc_as_source(model: LVCModel, name: Optional[str] = None) -> SourceModel:
    """The same linear-vibronic Hamiltonian written as a supplied potential:
    V(q) = V0 + sum_j q_j K_j + I sum_j m_j w_j^2 q_j^2 / 2, with the
    parameters [V0 slots (T), K_j slots (M x T), m_j w_j^2 (M)]."""
    n, M = model.n_states, model.n_modes
    T = n * (n + 1) // 2
    slots = [(k, l) for k in range(n) for l in range(k, n)]
    params = [model.v0[k, l] for k, l in slots]
    for j in range(M):
        params += [model.k[j, k, l] for k, l in slots]
    params += list(model.mass * model.omega ** 2)
    diag = ", ".join("1" if k == l else "0" for k, l in slots)
    hip = f"""
// binary64 and binary32 (templates): the binary32 kernels are built too
#define QCL_SOURCE_FP32 1
#define LVC_T {T}
__device__ constexpr int lvc_diag[LVC_T] = {{{diag}}};
template <typename T>
__device__ inline T lvc_k(int j, int s) {{ return (T)qcl_param[LVC_T * (1 + j) + s]; }}
template <typename T>
__device__ inline T lvc_mw2(int j) {{ return (T)qcl_param[LVC_T * (1 + QCL_M) + j]; }}
template <typename T>
__device__ void qcl_potential(const T *q, T *V)
{{
    T h = T(0);
    for (int j = 0; j < QCL_M; ++j)
        h += T(0.5) * lvc_mw2<T>(j) * q[j] * q[j];
    for (int s = 0; s < LVC_T; ++s) {{
        T v = (T)qcl_param[s];
        for (int j = 0; j < QCL_M; ++j)
            v += q[j] * lvc_k<T>(j, s);
        V[s] = lvc_diag[s] ? v + h : v;
    }}
}}
template <typename T>
__device__ void qcl_force(const T *q, const T *w, T *f)
{{
    T wd = T(0);
    for (int s = 0; s < LVC_T; ++s)
        wd += lvc_diag[s] ? w[s] : T(0);
    for (int j = 0; j < QCL_M; ++j) {{
        T g = lvc_mw2<T>(j) * q[j] * wd;
        for (int s = 0; s < LVC_T; ++s)
            g += w[s] * lvc_k<T>(j, s);
        f[j] = -g;
    }}
}}
template <typename T>
__device__ void qcl_coupling(const T *q, const T *v, T *K)
{{
    T h = T(0);
    for (int j = 0; j < QCL_M; ++j)
        h += v[j] * lvc_mw2<T>(j) * q[j];
    for (int s = 0; s < LVC_T; ++s) {{
        T k = T(0);
        for (int j = 0; j < QCL_M; ++j)
            k += v[j] * lvc_k<T>(j, s);
        K[s] = lvc_diag[s] ? k + h : k;
    }}
}}
"""
    c = f"""
#define LVC_N {n}
#define LVC_M {M}
#define LVC_T {T}
static int lvc_slot(int k, int l)
{{
    if (k > l) {{ int t = k; k = l; l = t; }}
    return k * LVC_N - k * (k - 1) / 2 + (l - k);
}}
void qcl_oracle_potential(const double *q, const double *prm, double *V)
{{
    double h = 0.0;
    for (int j = 0; j < LVC_M; ++j)
        h += 0.5 * prm[LVC_T * (1 + LVC_M) + j] * q[j] * q[j];
    for (int k = 0; k < LVC_N; ++k)
        for (int l = 0; l < LVC_N; ++l) {{
            int s = lvc_slot(k, l);
            double v = prm[s];
            for (int j = 0; j < LVC_M; ++j)
                v += q[j] * prm[LVC_T * (1 + j) + s];
            V[k * LVC_N + l] = (k == l) ? v + h : v;
        }}
}}
void qcl_oracle_gradient(int j, const double *q, const double *prm, double *G)
{{
    for (int k = 0; k < LVC_N; ++k)
        for (int l = 0; l < LVC_N; ++l) {{
            double g = prm[LVC_T * (1 + j) + lvc_slot(k, l)];
            G[k * LVC_N + l] = (k == l) ? g + prm[LVC_T * (1 + LVC_M) + j] * q[j] : g;
        }}
}}
"""
    return SourceModel(name=name or model.name + "_source", n_states_=n, mass=model.mass, omega=model.omega,
                       params=params, hip_source=hip, c_source=c, hbar=model.hbar, time_unit_fs=model.time_unit_fs)


def batched_instances(n_instances: int = 256, key: int = 4, **kw) -> List[Workload]:
    return [random_lvc(i, key=key, **kw) for i in range(n_instances)]


def served_stream(n_jobs: int = 200, rate: float = 20.0, seed: int = 5, traj_range=(1e5, 1e8),
                  max_modes: int = 100, steps_range=(500, 2000), traj_scale: float = 1.0,
                  step_scale: float = 1.0):
    """A job stream for the server: Poisson arrivals at ``rate`` jobs/s; each
    job is, with equal odds, the one-mode spin-boson run, the 3-mode Ohmic
    spin-boson run at kT 0.2, the same at kT 1.0, the pyrazine-like
    conical-intersection run, or an N-state (2-4) harmonic model with M
    log-uniform over [1, ``max_modes``], walkers log-uniform over
    ``traj_range`` and steps uniform over ``steps_range``.  Walker and step
    counts are multiplied by ``traj_scale`` and ``step_scale`` (small
    streams for tests).  Returns (arrival times, workloads)."""
    rng = np.random.Generator(np.random.Philox(key=[seed, 0]))
    t, arrivals, jobs = 0.0, [], []
    for i in range(n_jobs):
        t += float(rng.exponential(1.0 / rate))
        kind = int(rng.integers(0, 5))
        if kind == 0:
            wl = spin_boson_1mode()
        elif kind == 1:
            wl = spin_boson_ohmic(kT=0.2)
        elif kind == 2:
            wl = spin_boson_ohmic(kT=1.0)
        elif kind == 3:
            wl = pyrazine_ci()
        else:
            m = int(round(math.exp(rng.uniform(0.0, math.log(max_modes)))))
            wl = random_lvc(i, key=seed + 1000, n_modes=max(1, min(max_modes, m)), traj_range=traj_range,
                            steps_range=steps_range, cadence=50)
        r = wl.run
        r.n_traj = max(1, int(round(r.n_traj * traj_scale)))
        r.n_steps = max(r.cadence, int(round(r.n_steps * step_scale)) // r.cadence * r.cadence)
        arrivals.append(t)
        jobs.append(wl)
    return arrivals, jobs


NAMED = {
    "spin_boson_1mode": spin_boson_1mode,
    "spin_boson_ohmic": spin_boson_ohmic,
    "pyrazine_ci": pyrazine_ci,
    "zero_coupling": zero_coupling,
    "uncoupled_harmonic": uncoupled_harmonic,
}
