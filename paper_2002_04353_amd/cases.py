"""Seeded synthetic workloads (input generation only).

Each case bundles a mesh from ``meshgen``, the physical parameters of the run
(time step, viscosity, free stream, motion law) and the initial fields.  No
solver arithmetic lives here; parameters such as the viscosity are derived from
the dimensionless groups the paper uses (Sec. V: Ma = u / sqrt(gamma T),
Re = rho u c / mu, Sr = h w / u, k = w c / (2 u)).

Workloads:
  uniform      periodic unit square, 2000 jittered vertices, sinusoidal mesh
               deformation (amplitude 0.05, period 200 steps), rho=1, T=1,
               Ma=0.5; a uniform flow must stay uniform (GCL, Sec. III.A).
               T=1 lies outside the D2Q9 range (zero rest weight), so this
               run amplifies round-off; the paper's own values below are the
               meaningful uniform-flow test.
  uniform_paper  the same mesh with the free-stream test's own values
               (Sec. V.A): T=0.2, Ma=0.2, amplitude 500/8000 of the box,
               t0 = 1.5 L / u.
  vortex       isentropic vortex (strength 5, radius L/10) advected along the
               diagonal at Ma=0.3 on a deforming periodic mesh, L=112, 50,176
               P2 nodes, Re_R = 100 (at Re_R = 1000 with strength 5 the
               unshifted D2Q9 model diverges: the local Mach number reaches
               about 1).
  plunge       NACA0012 (chord 200) in an O-mesh of radius 20 chords, ~200k P2
               nodes, first spacing 0.5; plunge h = 0.2c, k = 1, Ma = 0.2,
               Re = 1e4.
  pitch        NACA0012, ~500k P2 nodes, first spacing 0.2; pitch 2.5 deg about
               c/4, k = 0.08, Ma = 0.76, Re = 5e6, blended to rest between 1.5c
               and 10c.
  ensemble     64 independent pitch+plunge NACA0012 cases, each on its own
               O-mesh of N ~ U(50k, 300k) P2 nodes (sum ~11M), Ma ~ U(0.2, 0.7),
               k ~ U(0.05, 1), pitch amplitude ~ U(0.5, 5) deg, plunge
               amplitude ~ U(0.02c, 0.25c), plunge phase ~ U(0, 2 pi),
               T = 0.3 and Re = 1850 (the paper's plunge values, Sec. V.B),
               deformation blended to rest between 1.5c and 10c.

Reynolds number and the trailing edge.  With the first spacing 0.5 and
dt = 0.125, Re = 1e4 puts the relaxation frequency near 1.8; there the method
(oracle and GPU alike) grows a cold, dense spot at the sharp trailing edge
after a few hundred steps (T falls towards 0.03 at constant pressure).  At the
paper's Re = 1850 the same meshes run without it, so the ensemble, whose runs
are long, uses Re = 1850; the single plunge workload keeps its stated Re = 1e4
for the short benchmark runs.

Time step.  The paper does not state dt.  The lattice velocities are |c_i| in
{0, 1, sqrt 2}; every case sets dt = CFL * h with h the smallest vertex
spacing (mean spacing on the periodic meshes, first-layer height on the
airfoil meshes) and CFL = 0.25.  At CFL near 1 the two-population BGK step is
linearly unstable on these meshes for relaxation frequencies above about 1.8
(measured on the oracle), while the interpolation at CFL 0.25 damps the grid
modes enough.
"""

from __future__ import annotations

import math
import os

import numpy as np

from . import meshgen

GAMMA = 1.4
PR = 0.71


def _sound(T):
    return math.sqrt(GAMMA * T)


CFL = 0.25  # dt |c| relative to the smallest vertex spacing (see the module docstring)


def _periodic_mesh(elem, nx, ny, Lx, Ly, seed, jitter=None):
    if elem == "p2":
        return meshgen.periodic_square(nx, ny, Lx, Ly, jitter=0.25 if jitter is None else jitter, seed=seed)
    if elem == "q2":
        return meshgen.periodic_square_quads(nx, ny, Lx, Ly, jitter=0.2 if jitter is None else jitter, seed=seed)
    raise ValueError(f"element kind {elem!r}: 'p2' or 'q2'")


def _airfoil_mesh(elem, n_nodes, chord, first, seed, **mesh_kw):
    """O-mesh of about n_nodes nodes: P2 triangles (``naca_omesh``) or 9-node
    quadrilaterals, structured at the wall (``naca_omesh_quads``)."""
    if elem == "p2":
        return meshgen.naca_omesh(n_nodes, chord=chord, first=first, seed=seed, **mesh_kw)
    if elem == "q2":
        return meshgen.naca_omesh_quads(n_nodes, chord=chord, first=first, seed=seed, **mesh_kw)
    raise ValueError(f"element kind {elem!r}: 'p2' or 'q2'")


# the smallest quadrilateral airfoil mesh (about 1e5 nodes): a coarser surface
# and two structured layers
SMALL_QUADS = dict(surface_ratio=4.0, structured_layers=2)


def uniform(nx=50, ny=40, seed=1, T=1.0, Ma=0.5, amp=0.05, period_steps=200, paper=False, elem="p2",
            jitter=None):
    m = _periodic_mesh(elem, nx, ny, 1.0, 1.0, seed, jitter)
    dt = CFL / math.sqrt(nx * ny)
    if paper:
        T, Ma, amp = 0.2, 0.2, 500.0 / 8000.0
    u = Ma * _sound(T)
    Tp = 1.5 * 1.0 / u if paper else period_steps * dt
    params = dict(gamma=GAMMA, Pr=PR, dt=dt, mu=0.5 * 1.0 * T * dt, rho_inf=1.0, u_inf=(u, 0.0),
                  T_inf=T, chord=1.0, ref_point=(0.0, 0.0), t0=0.0, motion="sine",
                  motion_p=[amp, 1.0, 1.0, Tp])
    N = m.n_nodes
    init = dict(rho=np.ones(N), ux=np.full(N, u), uy=np.zeros(N), T=np.full(N, T))
    steps = int(round(1.0 / (u * dt))) if paper else 200
    return dict(name="uniform_paper" if paper else "uniform", mesh=m, params=params, init=init,
                steps=steps)


def vortex_fields(x, y, t, L, U, R, beta, T_inf, rho_inf=1.0, gamma=GAMMA):
    """Isentropic vortex translated by U t on the periodic box (velocities in
    units of sqrt(T_inf)); returns rho, ux, uy, T at physical points."""
    xc = np.mod(0.5 * L + U[0] * t, L)
    yc = np.mod(0.5 * L + U[1] * t, L)
    dx = np.mod(x - xc + 0.5 * L, L) - 0.5 * L
    dy = np.mod(y - yc + 0.5 * L, L) - 0.5 * L
    xr, yr = dx / R, dy / R
    r2 = xr * xr + yr * yr
    e = np.exp(0.5 * (1.0 - r2))
    s = math.sqrt(T_inf)
    ux = U[0] - beta / (2 * math.pi) * e * yr * s
    uy = U[1] + beta / (2 * math.pi) * e * xr * s
    Tr = 1.0 - (gamma - 1.0) * beta**2 * np.exp(1.0 - r2) / (8.0 * gamma * math.pi**2)
    T = T_inf * Tr
    rho = rho_inf * Tr ** (1.0 / (gamma - 1.0))
    return rho, ux, uy, T


def vortex(n=112, L=112.0, seed=2, beta=5.0, Ma=0.3, T_inf=0.3, Re_R=100.0, amp_frac=0.05,
           period_steps=800, dt=None, steps=2000, elem="p2"):
    m = _periodic_mesh(elem, n, n, L, L, seed)
    if dt is None:
        dt = CFL * L / n
    Umag = Ma * _sound(T_inf)
    U = (Umag / math.sqrt(2.0), Umag / math.sqrt(2.0))
    R = L / 10.0
    mu = 1.0 * Umag * R / Re_R
    params = dict(gamma=GAMMA, Pr=PR, dt=dt, mu=mu, rho_inf=1.0, u_inf=U, T_inf=T_inf, chord=R,
                  ref_point=(0.0, 0.0), t0=0.0, motion="sine" if amp_frac > 0 else "none",
                  motion_p=[amp_frac * L, L, L, period_steps * dt])
    rho, ux, uy, T = vortex_fields(m.X[:, 0], m.X[:, 1], 0.0, L, U, R, beta, T_inf)
    init = dict(rho=rho, ux=ux, uy=uy, T=T)
    return dict(name="vortex", mesh=m, params=params, init=init, steps=steps,
                vortex=dict(L=L, U=U, R=R, beta=beta, T_inf=T_inf))


def _airfoil_params(chord, Ma, T_inf, Re):
    u = Ma * _sound(T_inf)
    mu = 1.0 * u * chord / Re
    return u, mu


def plunge(n_nodes=200_000, seed=3, first=0.5, chord=200.0, h_c=0.2, k=1.0, Ma=0.2, T_inf=0.3,
           Re=1e4, steps=1000, elem="p2", mesh_kw=None):
    m = _airfoil_mesh(elem, n_nodes, chord, first, seed, **(mesh_kw or {}))
    u, mu = _airfoil_params(chord, Ma, T_inf, Re)
    w = 2.0 * k * u / chord
    params = dict(gamma=GAMMA, Pr=PR, dt=CFL * first, mu=mu, rho_inf=1.0, u_inf=(u, 0.0), T_inf=T_inf,
                  chord=chord, ref_point=(0.25 * chord, 0.0), t0=0.0, motion="plunge",
                  motion_p=[h_c * chord, w, 0.0])
    N = m.n_nodes
    init = dict(rho=np.ones(N), ux=np.full(N, u), uy=np.zeros(N), T=np.full(N, T_inf))
    return dict(name="plunge", mesh=m, params=params, init=init, steps=steps)


def pitch(n_nodes=500_000, seed=4, first=0.2, chord=200.0, A_deg=2.5, k=0.08, Ma=0.76, T_inf=0.3,
          Re=5e6, h_c=0.0, phase_h=0.0, r0_c=1.5, r1_c=10.0, steps=1000, elem="p2", mesh_kw=None):
    m = _airfoil_mesh(elem, n_nodes, chord, first, seed, **(mesh_kw or {}))
    u, mu = _airfoil_params(chord, Ma, T_inf, Re)
    w = 2.0 * k * u / chord
    params = dict(gamma=GAMMA, Pr=PR, dt=CFL * first, mu=mu, rho_inf=1.0, u_inf=(u, 0.0), T_inf=T_inf,
                  chord=chord, ref_point=(0.25 * chord, 0.0), t0=0.0, motion="pitch_plunge",
                  motion_p=[math.radians(A_deg), w, 0.25 * chord, 0.0, 0.0, h_c * chord, phase_h,
                            r0_c * chord, r1_c * chord])
    N = m.n_nodes
    init = dict(rho=np.ones(N), ux=np.full(N, u), uy=np.zeros(N), T=np.full(N, T_inf))
    return dict(name="pitch", mesh=m, params=params, init=init, steps=steps)


ENSEMBLE_RANGES = dict(Ma=(0.2, 0.7), k=(0.05, 1.0), A_deg=(0.5, 5.0), h_c=(0.02, 0.25),
                       phase_h=(0.0, 2.0 * math.pi))


def _ensemble_mesh(arg):
    n, seed, cache_dir = arg
    path = os.path.join(cache_dir, f"naca_omesh_{n}_{seed}.npz") if cache_dir else None
    if path and os.path.exists(path):
        return meshgen.Mesh.load(path)
    m = meshgen.naca_omesh(n, chord=200.0, first=0.5, seed=seed)
    if path:
        tmp = path + ".tmp.npz"
        np.savez(tmp, n_vertices=m.n_vertices, **m.arrays())
        os.replace(tmp, path)
    return m


def pitch_plunge_params(Ma, k, A_deg, h_c, phase_h, T_inf=0.3, Re=1850.0, chord=200.0, first=0.5):
    """Solver parameters of one pitch+plunge case (Sec. V.C motion with a plunge,
    blended to rest between 1.5c and 10c) and its uniform initial state."""
    u, mu = _airfoil_params(chord, Ma, T_inf, Re)
    w = 2.0 * k * u / chord
    params = dict(gamma=GAMMA, Pr=PR, dt=CFL * first, mu=mu, rho_inf=1.0, u_inf=(u, 0.0), T_inf=T_inf,
                  chord=chord, ref_point=(0.25 * chord, 0.0), t0=0.0, motion="pitch_plunge",
                  motion_p=[math.radians(A_deg), w, 0.25 * chord, 0.0, 0.0, h_c * chord, phase_h,
                            1.5 * chord, 10.0 * chord])
    return params, u


def ensemble(n_cases=64, seed=11, n_min=50_000, n_max=300_000, T_inf=0.3, Re=1850.0, workers=1,
             cache_dir=None, shared_mesh=False, start_method="fork"):
    """Seeded batch of pitch+plunge cases on meshes of uneven size.

    Returns dict(name, meshes, params, inits, motion): one mesh, params dict and
    initial-field dict per case, and the five motion parameters of every case
    as an array [n_cases, 5] = (Ma, k, A_deg, h_c, phase_h).  ``workers`` > 1
    builds the meshes in a process pool: forked (call it before any GPU use) or,
    with ``start_method="spawn"``, fresh interpreters (safe at any time);
    ``cache_dir`` keeps each mesh as an .npz file there and reuses it.
    ``shared_mesh`` gives every case the same mesh of n_min nodes."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_min, n_max + 1, size=n_cases)
    draws = np.stack([rng.uniform(*ENSEMBLE_RANGES[k], size=n_cases)
                      for k in ("Ma", "k", "A_deg", "h_c", "phase_h")], axis=1)
    if cache_dir:
        os.makedirs(cache_dir, exist_ok=True)
    if shared_mesh:
        meshes = [_ensemble_mesh((int(n_min), 1000 * seed, cache_dir))] * n_cases
    else:
        args = [(int(sizes[c]), 1000 * seed + c, cache_dir) for c in range(n_cases)]
        if workers > 1:
            import multiprocessing as mp
            with mp.get_context(start_method).Pool(workers) as pool:
                meshes = pool.map(_ensemble_mesh, args)
        else:
            meshes = [_ensemble_mesh(a) for a in args]
    params, inits = [], []
    for c, m in enumerate(meshes):
        prm, u = pitch_plunge_params(*draws[c], T_inf=T_inf, Re=Re)
        params.append(prm)
        N = m.n_nodes
        inits.append(dict(rho=np.ones(N), ux=np.full(N, u), uy=np.zeros(N), T=np.full(N, T_inf)))
    return dict(name="ensemble", meshes=meshes, params=params, inits=inits, motion=draws)


def concat_init(inits):
    """Initial fields of a batch: the cases' node arrays concatenated in order."""
    return {k: np.concatenate([np.broadcast_to(i[k], (len(i["rho"]),)) for i in inits]) for k in inits[0]}


def small(name: str, **kw):
    """Reduced versions of the workloads for CPU tests and parity checks."""
    elem = kw.get("elem", "p2")
    if name == "uniform":
        return uniform(nx=kw.get("nx", 20), ny=kw.get("ny", 16), seed=kw.get("seed", 1), elem=elem)
    if name == "vortex":
        n = kw.get("n", 28)
        return vortex(n=n, L=float(n), seed=kw.get("seed", 2), beta=kw.get("beta", 5.0),
                      steps=kw.get("steps", 50), elem=elem)
    if name == "plunge":
        return plunge(n_nodes=kw.get("n_nodes", 20_000), seed=kw.get("seed", 3),
                      steps=kw.get("steps", 50), elem=elem, mesh_kw=SMALL_QUADS if elem == "q2" else None)
    if name == "pitch":
        return pitch(n_nodes=kw.get("n_nodes", 20_000), seed=kw.get("seed", 4), first=0.5,
                     steps=kw.get("steps", 50), elem=elem, mesh_kw=SMALL_QUADS if elem == "q2" else None)
    raise KeyError(name)


FULL = {"uniform": uniform, "uniform_paper": lambda: uniform(paper=True), "vortex": vortex,
        "plunge": plunge, "pitch": pitch, "ensemble": ensemble}
