"""FP64 CPU oracle of the 1D3V PIC-MCC step -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It wraps ``liboracle.so`` (plain C, built from
``pic_oracle.c`` by :func:`build`) and shares no code with the GPU library.
``oracle.mlp`` is the FP64 reference of the warm-start network.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MAX_SPECIES = 4
MAX_CHAN = 8
EEPF_BINS = 256


def build(force=True):
    """Compile the oracle with gcc (plain C99, no fast-math, no contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-ffp-contract=off", "-fopenmp",
                           "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


class Species(C.Structure):
    _fields_ = [("charge", C.c_double), ("mass", C.c_double), ("weight", C.c_double),
                ("capacity", C.c_int64), ("n_init", C.c_int64), ("vth", C.c_double),
                ("drift", C.c_double * 3), ("load", C.c_int32), ("pad", C.c_int32)]


class Config(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("bc", C.c_int32), ("field_solve", C.c_int32),
                ("n_species", C.c_int32), ("length", C.c_double), ("dt", C.c_double),
                ("eps0", C.c_double), ("rho_bg", C.c_double), ("e_unit", C.c_double),
                ("v_amp", C.c_double), ("v_freq", C.c_double), ("v_phase", C.c_double),
                ("e_ext", C.c_double * 3), ("b_ext", C.c_double * 3),
                ("gas_density", C.c_double), ("gas_temp", C.c_double),
                ("gas_mass", C.c_double), ("see_gamma", C.c_double),
                ("see_temp", C.c_double), ("perturb_eps", C.c_double),
                ("perturb_mode", C.c_int32), ("pad", C.c_int32), ("seed", C.c_uint64),
                ("sp", Species * MAX_SPECIES), ("renew_lz", C.c_double),
                ("drive", C.c_int32), ("waveform", C.c_int32), ("cap", C.c_double), ("j_amp", C.c_double)]


class Counters(C.Structure):
    _fields_ = [("absorbed", (C.c_int64 * 2) * MAX_SPECIES), ("see_emitted", C.c_int64 * 2),
                ("candidates", C.c_int64 * MAX_SPECIES), ("nulls", C.c_int64 * MAX_SPECIES),
                ("coll", (C.c_int64 * MAX_CHAN) * MAX_SPECIES),
                ("violations", C.c_int64 * MAX_SPECIES), ("dropped", C.c_int64),
                ("wall_energy", (C.c_double * 2) * MAX_SPECIES),
                ("renewed", C.c_int64 * MAX_SPECIES)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        up = C.POINTER(C.c_uint32)
        L.orc_create.argtypes = [C.POINTER(Config), C.POINTER(P)]
        L.orc_free.argtypes = [P]
        L.orc_free.restype = None
        L.orc_load_xsec.argtypes = [P, C.c_int32, C.c_int32, C.c_double, C.c_int32, dp, dp]
        L.orc_load.argtypes = [P]
        L.orc_get_moments.argtypes = [P, C.c_int32, dp, dp]
        L.orc_load_profiles.argtypes = [P, C.c_int32, dp, dp, C.POINTER(C.c_int64)]
        L.orc_set_particles.argtypes = [P, C.c_int32, C.c_int64, dp, dp, dp, dp, up, C.c_uint32]
        L.orc_get_particles.argtypes = [P, C.c_int32, C.c_int64, dp, dp, dp, dp, up,
                                        C.POINTER(C.c_int64), C.POINTER(C.c_uint32)]
        L.orc_set_axial.argtypes = [P, C.c_int32, C.c_int64, dp]
        L.orc_get_circuit.argtypes = [P, dp]
        L.orc_set_circuit.argtypes = [P, C.c_double]
        L.orc_get_axial.argtypes = [P, C.c_int32, C.c_int64, dp]
        L.orc_set_step.argtypes = [P, C.c_uint64]
        L.orc_get_power.argtypes = [P, C.c_int32, dp]
        L.orc_set_threads.argtypes = [P, C.c_int32]
        L.orc_get_step.argtypes = [P]
        L.orc_get_step.restype = C.c_uint64
        L.orc_refresh_field.argtypes = [P]
        L.orc_step.argtypes = [P, C.c_int32]
        L.orc_poisson.argtypes = [P, C.c_double, dp, dp, dp]
        L.orc_n_nodes.argtypes = [P]
        L.orc_get_field.argtypes = [P, dp, dp, dp]
        L.orc_get_density.argtypes = [P, C.c_int32, dp]
        L.orc_get_counters.argtypes = [P, C.POINTER(Counters)]
        L.orc_get_energy.argtypes = [P, dp, dp]
        L.orc_get_numax.argtypes = [P, C.c_int32, dp, up]
        L.orc_set_diag.argtypes = [P, C.c_int32, C.c_double]
        L.orc_set_wall_edf.argtypes = [P, C.c_int32, C.c_double]
        L.orc_reset_avg.argtypes = [P]
        L.orc_get_avg.argtypes = [P, dp]
        L.orc_get_eepf.argtypes = [P, dp]
        L.orc_get_wall_edf.argtypes = [P, dp]
        L.orc_philox4x32_10.argtypes = [up, up, up]
        L.orc_philox4x32_10.restype = None
        L.orc_u01.argtypes = [C.c_uint32]
        L.orc_u01.restype = C.c_double
        L.orc_boris.argtypes = [dp, dp, dp, C.c_double, C.c_double]
        L.orc_boris.restype = None
        L.orc_rotate.argtypes = [dp, C.c_double, C.c_double, dp]
        L.orc_rotate.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _up(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what} failed with status {code}")
        self.code = code


def _check(rc, what):
    if rc != 0:
        raise OracleError(rc, what)


def make_config(cfg):
    c = Config()
    c.n_cells = cfg["n_cells"]
    c.bc = cfg["bc"]
    c.field_solve = cfg["field_solve"]
    c.n_species = len(cfg["species"])
    for k in ("length", "dt", "eps0", "rho_bg", "e_unit", "v_amp", "v_freq", "v_phase",
              "gas_density", "gas_temp", "gas_mass", "see_gamma", "see_temp", "perturb_eps"):
        setattr(c, k, float(cfg[k]))
    for i in range(3):
        c.e_ext[i] = cfg["e_ext"][i]
        c.b_ext[i] = cfg["b_ext"][i]
    c.perturb_mode = cfg["perturb_mode"]
    c.seed = cfg["seed"]
    c.renew_lz = float(cfg.get("renew_lz", 0.0))
    c.drive = int(cfg.get("drive", 0))
    c.waveform = int(cfg.get("waveform", 0))
    c.cap = float(cfg.get("cap", 0.0))
    c.j_amp = float(cfg.get("j_amp", 0.0))
    for i, sp in enumerate(cfg["species"]):
        s = c.sp[i]
        s.charge, s.mass, s.weight = sp["charge"], sp["mass"], sp["weight"]
        s.capacity, s.n_init, s.vth = sp["capacity"], sp["n_init"], sp["vth"]
        for j in range(3):
            s.drift[j] = sp["drift"][j]
        s.load = sp["load"]
    return c


class Oracle:
    """One simulated discharge held by the C oracle."""

    def __init__(self, cfg, tables=(), load=True):
        self.cfg = cfg
        self._cfg = make_config(cfg)
        h = C.c_void_p()
        _check(lib().orc_create(C.byref(self._cfg), C.byref(h)), "orc_create")
        self.h = h
        self.n_species = len(cfg["species"])
        for t in tables:
            self.load_xsec(t["species"], t["kind"], t["threshold"], t["energy"], t["sigma"])
        if load:
            _check(lib().orc_load(self.h), "orc_load")

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_free(self.h)
            self.h = None

    def load_xsec(self, species, kind, threshold, energy, sigma):
        e = np.ascontiguousarray(energy, dtype=np.float64)
        s = np.ascontiguousarray(sigma, dtype=np.float64)
        _check(lib().orc_load_xsec(self.h, species, kind, threshold, len(e), _dp(e), _dp(s)),
               "orc_load_xsec")

    @property
    def n_nodes(self):
        return lib().orc_n_nodes(self.h)

    @property
    def step_index(self):
        return lib().orc_get_step(self.h)

    def set_step(self, n):
        _check(lib().orc_set_step(self.h, n), "orc_set_step")

    def set_threads(self, n):
        """0: the sequential step (default); n > 0: the parallel step on n
        threads, the same result for every n."""
        _check(lib().orc_set_threads(self.h, int(n)), "orc_set_threads")

    def step(self, n=1):
        _check(lib().orc_step(self.h, n), "orc_step")

    def load_profiles(self, density, temp_ev, n):
        """Replace every species by particles drawn from profiles [S][m]
        (density, temperature in eV) with n[s] particles each."""
        dens = np.ascontiguousarray(density, dtype=np.float64)
        temp = np.ascontiguousarray(temp_ev, dtype=np.float64)
        nn = (C.c_int64 * len(n))(*[int(v) for v in n])
        _check(lib().orc_load_profiles(self.h, dens.shape[1], _dp(dens), _dp(temp), nn), "orc_load_profiles")

    def moments(self, s):
        """(flux, x-momentum flux) densities of species s at the nodes."""
        n = self.n_nodes
        f, m = np.zeros(n), np.zeros(n)
        _check(lib().orc_get_moments(self.h, s, _dp(f), _dp(m)), "orc_get_moments")
        return f, m

    def refresh_field(self):
        _check(lib().orc_refresh_field(self.h), "orc_refresh_field")

    def get_particles(self, s):
        n = C.c_int64()
        nid = C.c_uint32()
        lib().orc_get_particles(self.h, s, 0, None, None, None, None, None, C.byref(n),
                                C.byref(nid))
        m = n.value
        x, vx, vy, vz = (np.zeros(m) for _ in range(4))
        ids = np.zeros(m, dtype=np.uint32)
        _check(lib().orc_get_particles(self.h, s, m, _dp(x), _dp(vx), _dp(vy), _dp(vz),
                                       _up(ids), C.byref(n), C.byref(nid)),
               "orc_get_particles")
        return dict(x=x, vx=vx, vy=vy, vz=vz, id=ids, next_id=nid.value)

    def set_particles(self, s, x, vx, vy, vz, ids, next_id=None):
        x, vx, vy, vz = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, vx, vy, vz))
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        if next_id is None:
            next_id = int(ids.max()) + 1 if len(ids) else 0
        _check(lib().orc_set_particles(self.h, s, len(x), _dp(x), _dp(vx), _dp(vy), _dp(vz),
                                       _up(ids), next_id), "orc_set_particles")

    def set_axial(self, s, z):
        """Axial displacements of species s (one per particle, canonical order)."""
        z = np.ascontiguousarray(z, dtype=np.float64)
        _check(lib().orc_set_axial(self.h, s, len(z), _dp(z)), "orc_set_axial")

    def axial(self, s):
        n = len(self.get_particles(s)["x"])
        z = np.zeros(n)
        _check(lib().orc_get_axial(self.h, s, n, _dp(z)), "orc_get_axial")
        return z

    def circuit(self):
        """(electrode potential at the last solve, the conductor's charge per area)."""
        o = np.zeros(2)
        _check(lib().orc_get_circuit(self.h, _dp(o)), "orc_get_circuit")
        return float(o[0]), float(o[1])

    def set_circuit(self, q):
        _check(lib().orc_set_circuit(self.h, float(q)), "orc_set_circuit")

    def field(self):
        n = self.n_nodes
        rho, phi, ef = np.zeros(n), np.zeros(n), np.zeros(n)
        _check(lib().orc_get_field(self.h, _dp(rho), _dp(phi), _dp(ef)), "orc_get_field")
        return rho, phi, ef

    def density(self, s):
        d = np.zeros(self.n_nodes)
        _check(lib().orc_get_density(self.h, s, _dp(d)), "orc_get_density")
        return d

    def poisson(self, t, rho):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        phi, ef = np.zeros(self.n_nodes), np.zeros(self.n_nodes)
        _check(lib().orc_poisson(self.h, t, _dp(rho), _dp(phi), _dp(ef)), "orc_poisson")
        return phi, ef

    def counters(self):
        c = Counters()
        _check(lib().orc_get_counters(self.h, C.byref(c)), "orc_get_counters")
        ns = self.n_species
        return dict(absorbed=np.array([[c.absorbed[k][w] for w in range(2)] for k in range(ns)]),
                    see_emitted=np.array([c.see_emitted[0], c.see_emitted[1]]),
                    candidates=np.array([c.candidates[k] for k in range(ns)]),
                    nulls=np.array([c.nulls[k] for k in range(ns)]),
                    coll=np.array([[c.coll[k][j] for j in range(MAX_CHAN)] for k in range(ns)]),
                    violations=np.array([c.violations[k] for k in range(ns)]),
                    dropped=c.dropped,
                    wall_energy=np.array([[c.wall_energy[k][w] for w in range(2)] for k in range(ns)]),
                    renewed=np.array([c.renewed[k] for k in range(ns)]))

    def set_diag(self, enable=True, eepf_emax=64.0):
        _check(lib().orc_set_diag(self.h, int(enable), float(eepf_emax)), "orc_set_diag")

    def power(self, s):
        """Time means of species s's power terms at the nodes: flux, momentum
        flux, q Gamma E, inertia, pressure, and the ohmic rest."""
        n = self.n_nodes
        o = np.zeros(5 * n)
        _check(lib().orc_get_power(self.h, s, _dp(o)), "orc_get_power")
        o = o.reshape(5, n)
        return dict(flux=o[0], momentum=o[1], power=o[2], inertia=o[3], pressure=o[4],
                    ohmic=o[2] - o[3] - o[4])

    def set_wall_edf(self, s, emax):
        _check(lib().orc_set_wall_edf(self.h, s, float(emax)), "orc_set_wall_edf")

    def reset_avg(self):
        _check(lib().orc_reset_avg(self.h), "orc_reset_avg")

    def avg(self):
        """Time means since the last reset: density per species, potential,
        electron mean energy (eV) at the nodes, and the number of samples."""
        S, n = self.n_species, self.n_nodes
        o = np.zeros(1 + (S + 2) * n)
        _check(lib().orc_get_avg(self.h, _dp(o)), "orc_get_avg")
        return dict(samples=o[0], density=o[1:1 + S * n].reshape(S, n),
                    phi=o[1 + S * n:1 + (S + 1) * n], mean_energy=o[1 + (S + 1) * n:])

    def eepf(self):
        o = np.zeros(2 * EEPF_BINS + 2)
        _check(lib().orc_get_eepf(self.h, _dp(o)), "orc_get_eepf")
        return dict(bulk=o[:EEPF_BINS], wall=o[EEPF_BINS:2 * EEPF_BINS],
                    bin_width=o[2 * EEPF_BINS], samples=o[2 * EEPF_BINS + 1])

    def wall_edf(self):
        """Impact-energy histograms [species][wall][bin], bin widths (eV) per
        species, samples."""
        S = self.n_species
        o = np.zeros(S * 2 * EEPF_BINS + S + 1)
        _check(lib().orc_get_wall_edf(self.h, _dp(o)), "orc_get_wall_edf")
        return dict(counts=o[:S * 2 * EEPF_BINS].reshape(S, 2, EEPF_BINS),
                    bin_width=o[S * 2 * EEPF_BINS:S * 2 * EEPF_BINS + S], samples=o[-1])

    def energy(self):
        ke = np.zeros(MAX_SPECIES)
        fe = C.c_double()
        _check(lib().orc_get_energy(self.h, _dp(ke), C.byref(fe)), "orc_get_energy")
        return ke[: self.n_species].copy(), fe.value

    def numax(self, s):
        nu = C.c_double()
        t = C.c_uint32()
        _check(lib().orc_get_numax(self.h, s, C.byref(nu), C.byref(t)), "orc_get_numax")
        return nu.value, t.value


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_up(c), _up(k), _up(out))
    return out


def u01(x):
    return lib().orc_u01(int(x))


def boris(v, e, b, qm, h):
    v = np.array(v, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    lib().orc_boris(_dp(v), _dp(e), _dp(b), qm, h)
    return v


def rotate(d, cos_chi, phi):
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_rotate(_dp(d), cos_chi, phi, _dp(out))
    return out
