"""Tiny hand-made systems for the oracle pins (test helper)."""
import numpy as np

from qsl_synth.gen import System


def make_tiny(shells, atoms, n_up, n_dn, T=30.0, seed=0):
    """shells: list of (atom, l, exps, raw_coefs)."""
    rng = np.random.default_rng(seed)
    sa = np.array([s[0] for s in shells], np.int32)
    sl = np.array([s[1] for s in shells], np.int32)
    sn = np.array([len(s[2]) for s in shells], np.int32)
    ex = np.concatenate([np.asarray(s[2], float) for s in shells])
    co = np.concatenate([np.asarray(s[3], float) for s in shells])
    return System(atom_xyz=np.asarray(atoms, float), atom_heavy=np.ones(len(atoms), bool),
                  shell_atom=sa, shell_l=sl, shell_nprim=sn, prim_exp=ex, prim_coef=co,
                  n_up=n_up, n_dn=n_dn, screen_T=T)


def random_tiny(n_atoms=2, n_up=3, n_dn=2, T=30.0, seed=0, lmax=2):
    """Small random system with s, p and d shells and square MO matrices."""
    rng = np.random.default_rng(seed)
    atoms = rng.normal(scale=1.5, size=(n_atoms, 3))
    shells = []
    for a in range(n_atoms):
        for l in range(lmax + 1):
            npr = int(rng.integers(1, 4))
            shells.append((a, l, np.exp(rng.uniform(np.log(0.2), np.log(8.0), npr)),
                           rng.uniform(0.1, 1.0, npr)))
    sysm = make_tiny(shells, atoms, n_up, n_dn, T=T)
    nb = sysm.n_basis
    A_up = rng.normal(size=(n_up, nb)) / np.sqrt(nb)
    A_dn = rng.normal(size=(n_dn, nb)) / np.sqrt(nb)
    return sysm, A_up, A_dn


def walkers_near(sysm, W, seed=1, sigma=0.8):
    rng = np.random.default_rng(seed)
    N = sysm.n_up + sysm.n_dn
    home = rng.integers(0, sysm.atom_xyz.shape[0], size=N)
    return sysm.atom_xyz[home][None] + rng.normal(scale=sigma, size=(W, N, 3))
