"""Seeded synthetic inputs for the ES-PIC workloads.

This module is shared by the GPU library's tests and by the CPU oracle's
tests.  It holds none of the method's arithmetic: it only writes down the
physical parameters of each workload and draws initial particle states and
drive waveforms from numpy's PCG64.  Both implementations derive their own
constants (q dt / m, collision thresholds, field scale factors) from the
parameters given here.

The paper's own data sets (the CCP benchmark of its Sec. 3.3, the 3D
breakdown runs of its Sec. 4.1) are not available; these generators stand in
for them with the same shapes: a 1D capacitively coupled argon discharge, a
static 2D quadtree refined inside a disk, a 2D electron avalanche ("streamer")
in a uniform field, a batched ensemble of 1D discharges and a served stream of
mixed jobs.
"""
from __future__ import annotations

import math

import numpy as np

# CODATA 2018
E_CHARGE = 1.602176634e-19
M_ELECTRON = 9.1093837015e-31
AMU = 1.66053906660e-27
K_BOLTZMANN = 1.380649e-23
TORR = 101325.0 / 760.0

MCC_NONE, MCC_ELECTRON, MCC_ION_CX = 0, 1, 2
WALL_NEUMANN, WALL_DIRICHLET = 0, 1
ABSORB, REFLECT = 0, 1
FIELD_CIC_EM, FIELD_CIC_EC = 0, 1   # 1D particle-field coupling (momentum- or energy-conserving CIC)
FIELD_DIPIC = 3                     # 1D: direct implicit PIC (D1 scheme, susceptibility in the Poisson solve)
FIELD_CIC_AMR = 2                   # 2D: cloud-in-cell on the quadtree (ghost cells at +-1 level)


def species(charge, mass, w0=1.0, mcc=MCC_NONE, sigma_el=0.0, sigma_iz=0.0, eps_iz=0.0,
            sigma_cx=0.0, eps_max=0.0):
    return dict(charge=float(charge), mass=float(mass), w0=float(w0), mcc=int(mcc),
                sigma_el=float(sigma_el), sigma_iz=float(sigma_iz), eps_iz=float(eps_iz),
                sigma_cx=float(sigma_cx), eps_max=float(eps_max))


# The largest position below 1 that stays below 1 in FP32 (a double in
# [1 - 2^-25, 1) rounds to 1.0 in FP32, outside the domain): normalised
# positions are drawn in [0, 1) and capped here, so the same inputs are
# valid at either particle precision.
S_MAX = 1.0 - 2.0 ** -24


def unit_positions(rng, shape):
    return np.minimum(rng.random(shape), S_MAX)


def base_desc(**kw):
    d = dict(dim=1, precision=64, length=1.0, dt=1e-12, ncells=0, min_level=0, max_level=0,
             base_level=0, refine_disk=0, disk_cx=0.5, disk_cy=0.5, disk_cz=0.5, disk_r=0.0, disk_level=0,
             field_bc=[WALL_NEUMANN] * 4, wall_phi=[0.0] * 4, particle_bc=ABSORB, depth_z=1.0,
             gas_density=0.0, gas_temperature=300.0, gas_mass=40.0 * AMU, seed=0, instance_key=0,
             species=[], field_scheme=FIELD_CIC_EM)
    d.update(kw)
    return d


# --------------------------------------------------------------------------
# 1D capacitively coupled discharge (argon), uniform mesh
# --------------------------------------------------------------------------
def ccp_desc(ncells=128, ppc=64, voltage=450.0, pressure_mtorr=30.0, precision=64, seed=1,
             instance_key=0, length=0.067, freq=13.56e6, steps_per_period=400, n0=1e14,
             te_ev=2.5, ti_ev=0.026, ion_amu=40.0, gas_temperature=300.0):
    dt = 1.0 / (steps_per_period * freq)
    n_g = pressure_mtorr * 1e-3 * TORR / (K_BOLTZMANN * gas_temperature)
    npart = ppc * ncells
    w0 = n0 * length / npart          # real particles per m^2 per computational particle
    m_i = ion_amu * AMU
    e = species(-E_CHARGE, M_ELECTRON, w0, MCC_ELECTRON, sigma_el=1e-19, sigma_iz=1e-20,
                eps_iz=15.8, eps_max=1000.0)
    i = species(E_CHARGE, m_i, w0, MCC_ION_CX, sigma_cx=5e-19, eps_max=1000.0)
    d = base_desc(dim=1, precision=precision, length=length, dt=dt, ncells=ncells,
                  particle_bc=ABSORB, gas_density=n_g, gas_temperature=gas_temperature,
                  gas_mass=m_i, seed=seed, instance_key=instance_key, species=[e, i])
    d["extra"] = dict(voltage=voltage, freq=freq, npart=npart, te_ev=te_ev, ti_ev=ti_ev,
                      ppc=ppc, pressure_mtorr=pressure_mtorr)
    return d


def dipic_ccp_desc(precision=64, n0=1e16, steps_per_period=200, **kw):
    """The 1D discharge at a hundred times the plasma density (n0 = 1e16
    m^-3) and twice the time step (200 steps per RF period): w_p dt = 2.08,
    where the explicit leapfrog is unstable, and dx = 4.4 Debye lengths at
    2.5 eV, beyond the explicit rule of about 3; stepped by the direct
    implicit scheme."""
    d = ccp_desc(precision=precision, n0=n0, steps_per_period=steps_per_period, **kw)
    d["field_scheme"] = FIELD_DIPIC
    return d


def maxwellian(rng, n, t_ev, mass):
    vth = math.sqrt(t_ev * E_CHARGE / mass)
    return rng.standard_normal((n, 3)) * vth


def ccp_particles(desc, rng_seed=None):
    """Uniform positions in (0,1) (normalised gap) and Maxwellian velocities.
    Returns [(s, v, w, id)] for electrons and ions; ids electrons first."""
    ex = desc["extra"]
    n = ex["npart"]
    rng = np.random.Generator(np.random.PCG64(desc["seed"] if rng_seed is None else rng_seed))
    out = []
    for k, (t_ev, sp) in enumerate(((ex["te_ev"], desc["species"][0]), (ex["ti_ev"], desc["species"][1]))):
        s = unit_positions(rng, n)
        v = maxwellian(rng, n, t_ev, sp["mass"])
        w = np.full(n, 65536, dtype=np.uint32)
        ids = np.arange(k * n, (k + 1) * n, dtype=np.uint32)
        out.append((s.reshape(n, 1), v, w, ids))
    return out


def drive_voltage(desc, n):
    """V(t_n) at the powered electrode x = 0, t_n = n dt (FP64 host)."""
    ex = desc["extra"]
    n = np.asarray(n, dtype=np.float64)
    return ex["voltage"] * np.sin(2.0 * math.pi * ex["freq"] * (n * desc["dt"]))


def ensemble_descs(count=96, seed=4, precision=32):
    """Batched ensemble: the 1D discharge's physics with per-instance mesh, ppc, voltage and
    pressure drawn from PCG64(seed): 'count' draws each of cells, ppc, V, p."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cells = np.exp(rng.uniform(math.log(128), math.log(4096), count))
    ppc = np.exp(rng.uniform(math.log(32), math.log(256), count))
    volt = rng.uniform(100.0, 600.0, count)
    pres = rng.uniform(10.0, 100.0, count)
    out = []
    for k in range(count):
        out.append(ccp_desc(ncells=int(round(cells[k])), ppc=int(round(ppc[k])), voltage=float(volt[k]),
                            pressure_mtorr=float(pres[k]), precision=precision, seed=seed, instance_key=k))
    return out


def ensemble_particles(desc):
    return ccp_particles(desc, rng_seed=[desc["seed"], desc["instance_key"]])


# --------------------------------------------------------------------------
# 2D static quadtree: base level 6, level 9 inside a centred disk
# --------------------------------------------------------------------------
def quadtree_static_desc(precision=32, seed=2):
    e = species(-E_CHARGE, M_ELECTRON, 1.0, MCC_NONE)
    return base_desc(dim=2, precision=precision, length=1.0, dt=1e-9, min_level=6, max_level=9,
                     base_level=6, refine_disk=1, disk_cx=0.5, disk_cy=0.5, disk_r=0.15, disk_level=9,
                     particle_bc=REFLECT, seed=seed, species=[e], gas_mass=40.0 * AMU)


def quadtree_particles(n, seed=2, t_ev=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    s = unit_positions(rng, (n, 2))
    v = maxwellian(rng, n, t_ev, M_ELECTRON)
    return s, v, np.full(n, 65536, dtype=np.uint32), np.arange(n, dtype=np.uint32)


def leaf_corners(keys, levels):
    """Physical-unit corner coordinates of leaves given (Morton key, level):
    returns x, y arrays of shape (nleaves, 4) in corner order (0,0),(1,0),(0,1),(1,1)."""
    keys = np.asarray(keys, dtype=np.uint64)
    lv = np.asarray(levels, dtype=np.int64)
    x = np.zeros(len(keys), dtype=np.uint64)
    y = np.zeros(len(keys), dtype=np.uint64)
    for b in range(16):
        x |= ((keys >> np.uint64(2 * b)) & np.uint64(1)) << np.uint64(b)
        y |= ((keys >> np.uint64(2 * b + 1)) & np.uint64(1)) << np.uint64(b)
    h = np.ldexp(1.0, -lv)
    x0 = x.astype(np.float64) / 65536.0
    y0 = y.astype(np.float64) / 65536.0
    cx = np.stack([x0, x0 + h, x0, x0 + h], axis=1)
    cy = np.stack([y0, y0, y0 + h, y0 + h], axis=1)
    return cx, cy


def quadtree_phi(x, y):
    """The static potential of the quadtree workload, V (x, y in m)."""
    return x * x + 0.3 * np.sin(2.0 * math.pi * y)


# --------------------------------------------------------------------------
# 3D static octree: base level 4 refined to level 7 inside a centred ball
# --------------------------------------------------------------------------
def octree_static_desc(precision=32, seed=7, base=4, top=7, r=0.15):
    e = species(-E_CHARGE, M_ELECTRON, 1.0, MCC_NONE)
    return base_desc(dim=3, precision=precision, length=1.0, dt=1e-9, min_level=base, max_level=top,
                     base_level=base, refine_disk=1, disk_cx=0.5, disk_cy=0.5, disk_cz=0.5, disk_r=r,
                     disk_level=top, particle_bc=REFLECT, seed=seed, species=[e], gas_mass=40.0 * AMU)


def octree_particles(n, seed=7, t_ev=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    s = unit_positions(rng, (n, 3))
    v = maxwellian(rng, n, t_ev, M_ELECTRON)
    return s, v, np.full(n, 65536, dtype=np.uint32), np.arange(n, dtype=np.uint32)


def leaf_corners3(keys, levels):
    """Physical-unit corner coordinates of octree leaves given (Morton key of
    the 10-bit corner coordinates, level): x, y, z arrays of shape
    (nleaves, 8), corner c = a + 2b + 4e along x, y, z."""
    keys = np.asarray(keys, dtype=np.uint64)
    lv = np.asarray(levels, dtype=np.int64)
    xyz = [np.zeros(len(keys), dtype=np.uint64) for _ in range(3)]
    for b in range(10):
        for a in range(3):
            xyz[a] |= ((keys >> np.uint64(3 * b + a)) & np.uint64(1)) << np.uint64(b)
    h = 2.0 ** (-lv.astype(np.float64))
    base = [x.astype(np.float64) / 1024.0 for x in xyz]
    out = []
    for a in range(3):
        side = np.array([(c >> a) & 1 for c in range(8)], dtype=np.float64)
        out.append(base[a][:, None] + side[None, :] * h[:, None])
    return out


def octree_phi(x, y, z):
    """The static potential of the octree workload, V (x, y, z in m)."""
    return x * x + 0.3 * np.sin(2.0 * math.pi * y) + 0.5 * z * z


def octree_avalanche_desc(precision=32, seed=8, side=0.005, e0=3e6, top=7):
    """Electron avalanche on a static octree in a uniform field along z
    (the avalanche physics above, 1 atm, 30 kV/cm), absorbing walls, levels
    4 to 7 refined around the seed."""
    n_g = 101325.0 / (K_BOLTZMANN * 300.0)
    m_i = 28.0 * AMU
    e = species(-E_CHARGE, M_ELECTRON, 1.0, MCC_ELECTRON, sigma_el=1e-19, sigma_iz=2e-20, eps_iz=15.6,
                eps_max=200.0)
    i = species(E_CHARGE, m_i, 1.0, MCC_NONE)
    d = base_desc(dim=3, precision=precision, length=side, dt=1e-13, min_level=4, max_level=top, base_level=4,
                  refine_disk=1, disk_cx=0.5, disk_cy=0.5, disk_cz=0.5, disk_r=0.2, disk_level=top,
                  particle_bc=ABSORB, gas_density=n_g, gas_temperature=300.0, gas_mass=m_i, seed=seed,
                  species=[e, i])
    d["extra"] = dict(e0=e0)
    return d


def octree_avalanche_phi(desc, x, y, z):
    """Potential of the uniform field along z: 0 at z = 0, E0 L at z = L."""
    return desc["extra"]["e0"] * z


def octree_avalanche_particles(desc, npairs=3000, sigma=0.1):
    rng = np.random.Generator(np.random.PCG64(desc["seed"]))
    pos = np.empty((0, 3))
    while len(pos) < npairs:
        p = rng.normal(0.5, sigma, size=(npairs, 3))
        p = p[np.all((p >= 0.0) & (p <= S_MAX), axis=1)]
        pos = np.concatenate([pos, p])[:npairs]
    ve = maxwellian(rng, npairs, 1.0, M_ELECTRON)
    vi = maxwellian(rng, npairs, K_BOLTZMANN * 300.0 / E_CHARGE, desc["species"][1]["mass"])
    w = np.full(npairs, 65536, dtype=np.uint32)
    return [(pos.copy(), ve, w.copy(), np.arange(npairs, dtype=np.uint32)),
            (pos.copy(), vi, w.copy(), np.arange(npairs, 2 * npairs, dtype=np.uint32))]


# --------------------------------------------------------------------------
# 2D avalanche / streamer in a uniform field on a dynamic quadtree
# --------------------------------------------------------------------------
def streamer_desc(side=0.01, precision=32, seed=3, e0=3e6, instance_key=0, min_level=5, max_level=11,
                  dt=1e-13, eps_max=200.0):
    n_g = 101325.0 / (K_BOLTZMANN * 300.0)
    m_i = 28.0 * AMU
    e = species(-E_CHARGE, M_ELECTRON, 1.0, MCC_ELECTRON, sigma_el=1e-19, sigma_iz=2e-20, eps_iz=15.6,
                eps_max=eps_max)
    i = species(E_CHARGE, m_i, 1.0, MCC_NONE)
    return base_desc(dim=2, precision=precision, length=side, dt=dt, min_level=min_level,
                     max_level=max_level, base_level=min_level,
                     field_bc=[WALL_NEUMANN, WALL_NEUMANN, WALL_DIRICHLET, WALL_DIRICHLET],
                     wall_phi=[0.0, 0.0, 0.0, e0 * side], particle_bc=ABSORB, depth_z=side,
                     gas_density=n_g, gas_temperature=300.0, gas_mass=m_i, seed=seed,
                     instance_key=instance_key, species=[e, i])


def streamer_particles(desc, npairs=10000, sigma=5e-4, rng_seed=None):
    """Gaussian seed of electron-ion pairs centred in the square; samples
    outside the domain are redrawn.  Electrons 1 eV, ions 300 K Maxwellian."""
    rng = np.random.Generator(np.random.PCG64(desc["seed"] if rng_seed is None else rng_seed))
    L = desc["length"]
    pos = np.empty((0, 2))
    while len(pos) < npairs:
        p = rng.normal(0.5, sigma / L, size=(npairs, 2))
        p = p[np.all((p >= 0.0) & (p <= S_MAX), axis=1)]
        pos = np.concatenate([pos, p])[:npairs]
    ve = maxwellian(rng, npairs, 1.0, M_ELECTRON)
    vi = maxwellian(rng, npairs, K_BOLTZMANN * 300.0 / E_CHARGE, desc["species"][1]["mass"])
    w = np.full(npairs, 65536, dtype=np.uint32)
    return [(pos.copy(), ve, w.copy(), np.arange(npairs, dtype=np.uint32)),
            (pos.copy(), vi, w.copy(), np.arange(npairs, 2 * npairs, dtype=np.uint32))]


def avalanche_ensemble(count=32, seed=6, precision=32):
    """Batched ensemble of 2D avalanches shaped like the served stream's 2D
    jobs: domain side uniform in 0.25-1 cm, seed pairs uniform in 1e3-1e4,
    the avalanche physics above (levels 5-11, 30 kV/cm), a Philox key and a
    seed draw of its own per instance.  Returns [(desc, particles)]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sides = rng.uniform(0.0025, 0.01, count)
    npairs = rng.integers(1000, 10001, count)
    out = []
    for k in range(count):
        d = streamer_desc(side=float(sides[k]), precision=precision, seed=seed, instance_key=k)
        out.append((d, streamer_particles(d, npairs=int(npairs[k]), rng_seed=[seed, k])))
    return out


# --------------------------------------------------------------------------
# Served request stream
# --------------------------------------------------------------------------
def job_stream(rate=20.0, duration=600.0, seed=5, frac_ccp=0.7):
    """Poisson arrivals; each job is a dict with its arrival time, kind, descriptor
    parameters and step count."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    jobs = []
    k = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        if rng.random() < frac_ccp:
            cells = int(round(math.exp(rng.uniform(math.log(128), math.log(4096)))))
            ppc = int(round(math.exp(rng.uniform(math.log(32), math.log(256)))))
            jobs.append(dict(arrival=t, kind="ccp", ncells=cells, ppc=ppc,
                             voltage=float(rng.uniform(100, 600)), pressure=float(rng.uniform(10, 100)),
                             steps=int(rng.integers(500, 5001)), key=k))
        else:
            jobs.append(dict(arrival=t, kind="streamer", side=float(rng.uniform(0.0025, 0.01)),
                             npairs=int(rng.integers(1000, 10001)), steps=2000, key=k))
        k += 1
    return jobs
