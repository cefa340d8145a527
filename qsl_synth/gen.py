"""Synthetic peptide-shaped molecular systems and QMC walker snapshots.

The paper benchmarks real molecules (a copper complex of 158 electrons, a
434-electron beta-strand, 1ZE7 with 1056 and 1AMB with 1731 electrons;
section "Exploiting the highly localized character of atomic basis
functions", Table 1).  Their geometries, basis sets, Hartree-Fock orbitals
and VMC samples are not available here, so these generators stand in for
them with the same electron counts and the same kind of structure:

* atoms placed as a self-avoiding random-walk chain (bond 2.8 bohr, minimum
  non-bonded distance 2.0 bohr), heavy atoms evenly interleaved with H;
* Cartesian contracted Gaussian shells (the AO form of the paper's
  equations for chi(r) and g(r)): heavy atom s,s,s,p,p,d (15 AOs),
  H s,s,p (5 AOs), 3 primitives per shell, exponents log-uniform in
  [0.1, 50], raw contraction weights uniform in [0.1, 1];
* dense MO coefficients a_ij ~ N(0,1)/sqrt(N_basis), independent per spin,
  rounded once to FP32 where the workload says FP32 coefficients;
* walkers: 6 electrons per heavy atom and 1 per H, each a Gaussian
  (sigma = 1 bohr) about its atom; even electron index = spin up, then a
  stable reorder puts the up electrons first (N_up = ceil(N/2)).

Only raw inputs are produced: the normalisation of the contraction weights
is part of the method and is done separately by the oracle and by the
library.
"""
from __future__ import annotations

import dataclasses
import numpy as np

BOND = 2.8          # bohr
MIN_DIST = 2.0      # bohr, self-avoidance of the chain
SCREEN_T = 30.0     # primitive k is kept iff gamma_k * r^2 <= T
HEAVY_SHELLS = (0, 0, 0, 1, 1, 2)
H_SHELLS = (0, 0, 1)
NPRIM = 3
EXP_LO, EXP_HI = 0.1, 50.0
HEAVY_ELECTRONS = 6


@dataclasses.dataclass
class System:
    atom_xyz: np.ndarray      # [n_atoms, 3] f64
    atom_heavy: np.ndarray    # [n_atoms] bool
    shell_atom: np.ndarray    # [n_shells] int32 (atom-major order)
    shell_l: np.ndarray       # [n_shells] int32
    shell_nprim: np.ndarray   # [n_shells] int32
    prim_exp: np.ndarray      # [sum nprim] f64
    prim_coef: np.ndarray     # [sum nprim] f64 raw (un-normalised) weights
    n_up: int
    n_dn: int
    screen_T: float = SCREEN_T

    @property
    def n_atoms(self) -> int:
        return int(self.atom_xyz.shape[0])

    @property
    def n_shells(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def n_elec(self) -> int:
        return self.n_up + self.n_dn

    @property
    def n_basis(self) -> int:
        # number of Cartesian components per shell: (l+1)(l+2)/2
        l = self.shell_l.astype(np.int64)
        return int(((l + 1) * (l + 2) // 2).sum())


# name -> (n_heavy, n_H, walkers, mode, fp32 MO coefficients, seed)
CONFIGS = {
    "44e": dict(n_heavy=6, n_h=8, W=64, mode="fp64", a_fp32=False, seed=1001),
    "158e": dict(n_heavy=22, n_h=26, W=1024, mode="fp32", a_fp32=True, seed=1002),
    "434e": dict(n_heavy=60, n_h=74, W=4096, mode="bf16x3", a_fp32=True, seed=1003),
    "1731e": dict(n_heavy=240, n_h=291, W=512, mode="fp32", a_fp32=True, seed=1005),
}


def _streams(seed: int):
    """Three independent PCG64 streams: geometry/basis, MOs, walkers."""
    ss = np.random.SeedSequence(seed)
    g, m, w = ss.spawn(3)
    return (np.random.Generator(np.random.PCG64(g)),
            np.random.Generator(np.random.PCG64(m)),
            np.random.Generator(np.random.PCG64(w)))


def atom_kinds(n_heavy: int, n_h: int) -> np.ndarray:
    """Atom i is heavy iff floor((i+1)h/n) > floor(i h/n): even interleave."""
    n = n_heavy + n_h
    i = np.arange(n)
    return ((i + 1) * n_heavy // n) > (i * n_heavy // n)


def chain_geometry(n: int, rng: np.random.Generator) -> np.ndarray:
    q = np.zeros((n, 3))
    for i in range(1, n):
        for _ in range(100000):
            u = rng.standard_normal(3)
            u /= np.linalg.norm(u)
            cand = q[i - 1] + BOND * u
            if i < 2 or np.min(np.linalg.norm(q[:i] - cand, axis=1)) >= MIN_DIST:
                break
        else:  # pragma: no cover - practically unreachable
            raise RuntimeError("self-avoiding walk got stuck")
        q[i] = cand
    return q


def make_system(n_heavy: int, n_h: int, seed: int, screen_T: float = SCREEN_T) -> System:
    rg, _, _ = _streams(seed)
    heavy = atom_kinds(n_heavy, n_h)
    xyz = chain_geometry(heavy.shape[0], rg)
    sa, sl = [], []
    for a, hv in enumerate(heavy):
        for l in (HEAVY_SHELLS if hv else H_SHELLS):
            sa.append(a)
            sl.append(l)
    ns = len(sl)
    exps = np.exp(rg.uniform(np.log(EXP_LO), np.log(EXP_HI), size=ns * NPRIM))
    coefs = rg.uniform(0.1, 1.0, size=ns * NPRIM)
    n_el = int(heavy.sum()) * HEAVY_ELECTRONS + int((~heavy).sum())
    n_up = (n_el + 1) // 2
    return System(atom_xyz=xyz, atom_heavy=heavy,
                  shell_atom=np.asarray(sa, np.int32), shell_l=np.asarray(sl, np.int32),
                  shell_nprim=np.full(ns, NPRIM, np.int32),
                  prim_exp=exps, prim_coef=coefs, n_up=n_up, n_dn=n_el - n_up,
                  screen_T=float(screen_T))


def make_mos(sys: System, seed: int, fp32: bool):
    """A^up [n_up, N_b] and A^dn [n_dn, N_b], row-major f64 (FP32-rounded if asked)."""
    _, rm, _ = _streams(seed)
    nb = sys.n_basis
    a_up = rm.standard_normal((sys.n_up, nb)) / np.sqrt(nb)
    a_dn = rm.standard_normal((sys.n_dn, nb)) / np.sqrt(nb)
    if fp32:
        a_up = a_up.astype(np.float32).astype(np.float64)
        a_dn = a_dn.astype(np.float32).astype(np.float64)
    return np.ascontiguousarray(a_up), np.ascontiguousarray(a_dn)


def electron_atoms(sys: System) -> np.ndarray:
    """Home atom of each electron in output order (ups first)."""
    home = []
    for a, hv in enumerate(sys.atom_heavy):
        home += [a] * (HEAVY_ELECTRONS if hv else 1)
    home = np.asarray(home)
    idx = np.arange(home.shape[0])
    order = np.concatenate([idx[idx % 2 == 0], idx[idx % 2 == 1]])
    return home[order]


def make_walkers(sys: System, W: int, seed: int) -> np.ndarray:
    """R [W, N, 3] f64; the first W' walkers do not depend on W."""
    _, _, rw = _streams(seed)
    home = electron_atoms(sys)
    noise = rw.standard_normal((W, home.shape[0], 3))
    return np.ascontiguousarray(sys.atom_xyz[home][None, :, :] + noise)


def make_config(name: str, W: int | None = None):
    c = CONFIGS[name]
    sys = make_system(c["n_heavy"], c["n_h"], c["seed"])
    a_up, a_dn = make_mos(sys, c["seed"], c["a_fp32"])
    R = make_walkers(sys, c["W"] if W is None else W, c["seed"])
    return sys, a_up, a_dn, R


def nuclear_charges(sys: System) -> np.ndarray:
    """Charges of the synthetic nuclei: a heavy atom carries the 6 electrons
    the walkers place around it, a hydrogen 1 (a neutral molecule)."""
    return np.where(sys.atom_heavy, 6.0, 1.0)


def dmc_randoms(W: int, N: int, seed: int, step: int):
    """Standard normal deviates eta [W, N, 3] and uniforms u [W] in [0, 1) of
    Monte Carlo step `step` (their own PCG64 stream per step)."""
    rng = np.random.Generator(np.random.PCG64([seed, 7919, step]))
    return rng.standard_normal((W, N, 3)), rng.random(W)


def localize_mos(sys: System, a_up: np.ndarray, a_dn: np.ndarray, radius: float):
    """Localised stand-ins for the MO coefficients: MO i of a spin keeps its
    coefficients on the AOs of atoms within `radius` bohr of the home atom of
    electron i of that spin and is zero elsewhere (MOs stay ordered along the
    chain, so the non-zeros form blocks).  Returns copies."""
    home = electron_atoms(sys)
    ao_atom = np.repeat(sys.shell_atom, (sys.shell_l + 1) * (sys.shell_l + 2) // 2)
    d = np.linalg.norm(sys.atom_xyz[:, None, :] - sys.atom_xyz[None, :, :], axis=2)
    out = []
    for a, centers in ((a_up, home[:sys.n_up]), (a_dn, home[sys.n_up:])):
        keep = d[centers][:, ao_atom] <= radius
        out.append(np.where(keep, a, 0.0))
    return out[0], out[1]
