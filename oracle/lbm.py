"""Lattice state, initial condition and time stepping (oracle; test infrastructure).

State at time n: pre-collision populations f (Q, N3, N2, N1) and phi
(P, N3, N2, N1), float64, full values (not deviations), index order
[population][z][y][x].

Boundaries (Sec. 2.5): half-way bounce-back for no-slip (f) and no-flux (phi)
at x = 0, x = N1 (end walls) and z = 0, z = N3 (bottom, top); the span y is
periodic. Streaming in pull form: f_q(x, n+1) = f*_q(x - c_q) when x - c_q is a
fluid node, else f*_opp(q)(x) (the population reflected at the wall half-way
between the node and its missing neighbour). Walls are at rest.

Initial state (Sec. 2.5): zero velocity (j = 0, f = w), chi0 = 1 inside the
lock (x-index i < lock_fraction * N1), 0 elsewhere, plus a seeded uniform
perturbation of amplitude a in the two columns next to the gate. The
perturbation's random numbers come from SplitMix64 (Steele, Lea and Flood,
2014), written out below from its published definition.
"""
import numpy as np
import torch

from . import collide as C
from .params import Config, derive  # noqa: F401  (re-exported for callers)

GOLDEN = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def splitmix64(x):
    """SplitMix64 output for state x (numpy uint64 array): add the golden
    gamma, then two xor-shift-multiply rounds and a final xor-shift."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over='ignore'):
        z = x + np.uint64(GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def gate_index(nx, lock_fraction):
    return int(np.floor(lock_fraction * nx))


def chi0_lock_exchange(cfg, lock_fraction=0.125, amp=1e-3, seed=0):
    """chi0 (N3, N2, N1) float64: step function plus noise a (2U - 1) in the
    columns i_gate - 1 and i_gate, U = (splitmix64(seed ^ l*gamma) >> 11) 2^-53
    with l = i + N1 (j + N2 k) the linear node index."""
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    ig = gate_index(nx, lock_fraction)
    chi = torch.zeros(nz, ny, nx, dtype=torch.float64)
    chi[:, :, :ig] = 1.0
    if amp != 0.0:
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing='ij')
        lin = (i + nx * (j + ny * k)).astype(np.uint64)
        with np.errstate(over='ignore'):
            key = np.uint64(seed & _M64) ^ (lin * np.uint64(GOLDEN))
        r = splitmix64(key)
        U = (r >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        eta = torch.from_numpy(amp * (2.0 * U - 1.0))
        for col in (ig - 1, ig):
            if 0 <= col < nx:
                chi[:, :, col] += eta[:, :, col]
    return chi


def init_state(P, chi0):
    """f = w (rest, j = 0), phi = w_phi chi0."""
    nz, ny, nx = chi0.shape
    f = P.flow.w[:, None, None, None].expand(P.flow.Q, nz, ny, nx).clone()
    phi = P.scal.w[:, None, None, None] * chi0[None]
    return f, phi


def stream(fs, lat, periodic_x=False, periodic_z=False):
    """Pull streaming with half-way bounce-back (x, z walls) and periodic y."""
    Q, nz, ny, nx = fs.shape
    out = []
    for q in range(Q):
        cx, cy, cz = lat.c_list[q]
        src = torch.roll(fs[q], shifts=(cz, cy, cx), dims=(0, 1, 2))
        wall = torch.zeros(nz, ny, nx, dtype=torch.bool)
        if not periodic_x and cx != 0:
            wall[:, :, 0 if cx == 1 else nx - 1] = True
        if not periodic_z and cz != 0:
            wall[0 if cz == 1 else nz - 1, :, :] = True
        out.append(torch.where(wall, fs[int(lat.opp[q])], src))
    return torch.stack(out)


def collide_field(f, phi, P, cs_smag=None, sc_t=None, chunk=1 << 15):
    """Apply the local collision at every node, in chunks of nodes."""
    Q = f.shape[0]
    Pq = phi.shape[0]
    shp = f.shape[1:]
    ff = f.reshape(Q, -1)
    pp = phi.reshape(Pq, -1)
    outs_f, outs_p = [], []
    for s in range(0, ff.shape[1], chunk):
        a, b = C.collide(ff[:, s:s + chunk], pp[:, s:s + chunk], P, cs_smag, sc_t)
        outs_f.append(a)
        outs_p.append(b)
    return torch.cat(outs_f, 1).reshape(Q, *shp), torch.cat(outs_p, 1).reshape(Pq, *shp)


def step(f, phi, P, cs_smag=None, sc_t=None):
    """One time step n -> n+1 (Eq. 17, 28): collide at every node, then stream."""
    fs, ps = collide_field(f, phi, P, cs_smag, sc_t)
    px, pz = P.cfg.periodic_x, P.cfg.periodic_z
    return stream(fs, P.flow, px, pz), stream(ps, P.scal, px, pz)


def run(f, phi, P, nsteps):
    for _ in range(nsteps):
        f, phi = step(f, phi, P)
    return f, phi


def moments(f, phi, P):
    """rho, u (3,...), chi of the pre-collision state (Eq. 19-20, 27)."""
    Q = f.shape[0]
    shp = f.shape[1:]
    rho, j, chi, F, u = C.macroscopic(f.reshape(Q, -1), phi.reshape(phi.shape[0], -1), P)
    return rho.reshape(shp), u.reshape(3, *shp), chi.reshape(shp)


def step_at(f, phi, P, nodes):
    """f(n+1), phi(n+1) at the listed nodes only ((k, j, i) integer triples),
    by colliding the nodes they pull from. Same definition as ``step``,
    restricted to a sample of nodes, for checks at sizes where a full oracle
    step is too slow. Returns (Q, m), (P, m)."""
    nz, ny, nx = f.shape[1:]
    cols = {}
    plans = ([], [])
    for which, lat in enumerate((P.flow, P.scal)):
        for m, (k, j, i) in enumerate(nodes):
            for q in range(lat.Q):
                cx, cy, cz = lat.c_list[q]
                sk, sj, si = k - cz, (j - cy) % ny, i - cx
                if P.cfg.periodic_x:
                    si %= nx
                if P.cfg.periodic_z:
                    sk %= nz
                if 0 <= si < nx and 0 <= sk < nz:
                    src, qq = (sk, sj, si), q
                else:
                    src, qq = (k, j, i), int(lat.opp[q])
                col = cols.setdefault(src, len(cols))
                plans[which].append((q, m, col, qq))
    ks = torch.tensor([c[0] for c in cols])
    js = torch.tensor([c[1] for c in cols])
    iis = torch.tensor([c[2] for c in cols])
    fs, ps = C.collide(f[:, ks, js, iis], phi[:, ks, js, iis], P)
    out_f = torch.empty(P.flow.Q, len(nodes), dtype=torch.float64)
    out_p = torch.empty(P.scal.Q, len(nodes), dtype=torch.float64)
    for (out, src), plan in zip(((out_f, fs), (out_p, ps)), plans):
        for q, m, col, qq in plan:
            out[q, m] = src[qq, col]
    return out_f, out_p
