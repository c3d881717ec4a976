"""Python binding of the MI355X PIC-MCC library (``libpic_mi355x.so``).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI of ``include/pic.h``.  PyTorch supplies device memory (through
the library's allocator hook, backed by torch's caching allocator) and the HIP
stream.  There is no CPU fallback: without the built library or a GPU the
constructor raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic_mi355x.so")
LIB_PATH = os.environ.get("PIC_MI355X_LIB", LIB_PATH)   # another build of the same library

MAX_SPECIES = 4
MAX_CHAN = 8
EEPF_BINS = 256

OK, EINVAL, ENOMEM, EHIP, ECAPACITY, ENUMERIC, ESTATE, ESTALL, ESCRATCH = 0, -1, -2, -3, -4, -5, -6, -7, -8
DIAG = dict(COUNTS=0, RHO=1, PHI=2, EFIELD=3, DENSITY=4, ENERGY=5, WALL=6, COLL=7, NUMAX=8,
            FLAGS=9, AVG=10, EEPF=11, RESET_AVG=12, CHARGE=13, TIMING=14, POWER=15, WALL_ENERGY=16, WALL_EDF=17, RENEWED=18, CIRCUIT=19, GRAPHS=20)


class SpeciesCfg(C.Structure):
    _fields_ = [("charge", C.c_double), ("mass", C.c_double), ("weight", C.c_double),
                ("capacity", C.c_int64), ("n_init", C.c_int64), ("vth", C.c_double),
                ("drift", C.c_double * 3), ("load", C.c_int32), ("pad", C.c_int32)]


class PicConfig(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("bc", C.c_int32), ("field_solve", C.c_int32),
                ("n_species", C.c_int32), ("length", C.c_double), ("dt", C.c_double),
                ("eps0", C.c_double), ("rho_bg", C.c_double), ("e_unit", C.c_double),
                ("v_amp", C.c_double), ("v_freq", C.c_double), ("v_phase", C.c_double),
                ("e_ext", C.c_double * 3), ("b_ext", C.c_double * 3),
                ("gas_density", C.c_double), ("gas_temp", C.c_double), ("gas_mass", C.c_double),
                ("see_gamma", C.c_double), ("see_temp", C.c_double), ("perturb_eps", C.c_double),
                ("perturb_mode", C.c_int32), ("pad", C.c_int32), ("seed", C.c_uint64),
                ("species", SpeciesCfg * MAX_SPECIES), ("renew_lz", C.c_double),
                ("drive", C.c_int32), ("waveform", C.c_int32), ("cap", C.c_double), ("j_amp", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class PicAllocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class PicError(RuntimeError):
    def __init__(self, code, what):
        msg = _lib.pic_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})")
        self.code = code


_lib = None
_live = []          # weak references to open contexts, closed before torch unloads


def _close_all():
    for r in list(_live):
        sim = r()
        if sim is not None:
            sim.close()


import atexit        # noqa: E402
import weakref       # noqa: E402

atexit.register(_close_all)


def load_library():
    """dlopen the built library and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2609_17151_amd/build.py")
    L = C.CDLL(LIB_PATH)
    P, i32, i64, u32, u64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
    dp, fp, ip, up = (C.POINTER(C.c_double), C.POINTER(C.c_float), C.POINTER(C.c_int32),
                      C.POINTER(C.c_uint32))
    sig = {
        "pic_init": (i32, [C.POINTER(PicConfig), i32, C.POINTER(PicAllocator), P, C.POINTER(P)]),
        "pic_load_xsec": (i32, [P, i32, i32, i32, d, i32, dp, dp]),
        "pic_step": (i32, [P, i32]),
        "pic_poisson": (i32, [P, i32, d, dp, dp, dp]),
        "pic_diag": (i32, [P, i32, i32, P, C.c_size_t]),
        "pic_get_particles": (i32, [P, i32, i32, i64, ip, fp, fp, fp, fp, up,
                                    C.POINTER(i64), C.POINTER(u32)]),
        "pic_set_particles": (i32, [P, i32, i32, i64, ip, fp, fp, fp, fp, up, u32, u64]),
        "pic_sync": (i32, [P]),
        "pic_strerror": (C.c_char_p, [i32]),
        "pic_free": (None, [P]),
        "pic_config_tiles": (i32, [P, i32, i32, i32, i32]),
        "pic_config_events": (i32, [P, i32]),
        "pic_thin": (i32, [P, i32, i64, i64]),
        "pic_set_diag": (i32, [P, i32, d]),
        "pic_set_wall_edf": (i32, [P, i32, d]),
        "pic_get_axial": (i32, [P, i32, i32, i64, dp, C.POINTER(i64)]),
        "pic_set_axial": (i32, [P, i32, i32, i64, dp]),
        "pic_set_circuit": (i32, [P, i32, d]),
        "pic_set_windows": (i32, [P, i32, i64]),
        "pic_get_windows": (i32, [P, i32, i64, i32, dp, C.POINTER(i64)]),
        "pic_profile": (i32, [P, i32]),
        "pic_use_graphs": (i32, [P, i32]),
        "pic_sort": (i32, [P]),
        "pic_sort_noalloc": (i32, [P]),
        "pic_retire": (i32, [P, i32, i32]),
        "pic_load_profiles": (i32, [P, i32, i32, dp, dp, C.POINTER(i64)]),
        "pic_mlp_create": (i32, [ip, i32, i32, C.POINTER(PicAllocator), P, C.POINTER(P)]),
        "pic_mlp_n_params": (i64, [P]),
        "pic_mlp_set_params": (i32, [P, fp, i64]),
        "pic_mlp_get_params": (i32, [P, fp, i64]),
        "pic_mlp_forward": (i32, [P, i32, P, P]),
        "pic_mlp_train_step": (i32, [P, i32, P, P, C.c_float, C.c_float, C.c_float, C.c_float, P]),
        "pic_mlp_grad": (i32, [P, i32, P, P, fp, fp]),
        "pic_mlp_sync": (i32, [P]),
        "pic_mlp_free": (None, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def make_config(cfg):
    c = PicConfig()
    c.n_cells, c.bc, c.field_solve = cfg["n_cells"], cfg["bc"], cfg["field_solve"]
    c.n_species = len(cfg["species"])
    for k in ("length", "dt", "eps0", "rho_bg", "e_unit", "v_amp", "v_freq", "v_phase",
              "gas_density", "gas_temp", "gas_mass", "see_gamma", "see_temp", "perturb_eps"):
        setattr(c, k, float(cfg[k]))
    for i in range(3):
        c.e_ext[i], c.b_ext[i] = cfg["e_ext"][i], cfg["b_ext"][i]
    c.perturb_mode, c.seed = cfg["perturb_mode"], cfg["seed"]
    c.renew_lz = float(cfg.get("renew_lz", 0.0))
    c.drive = int(cfg.get("drive", 0))
    c.waveform = int(cfg.get("waveform", 0))
    c.cap = float(cfg.get("cap", 0.0))
    c.j_amp = float(cfg.get("j_amp", 0.0))
    for i, sp in enumerate(cfg["species"]):
        s = c.species[i]
        s.charge, s.mass, s.weight = sp["charge"], sp["mass"], sp["weight"]
        s.capacity, s.n_init, s.vth = sp["capacity"], sp["n_init"], sp["vth"]
        for j in range(3):
            s.drift[j] = sp["drift"][j]
        s.load = sp["load"]
    return c


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class Sim:
    """A batch of discharges on one GPU (``pic_ctx``)."""

    def __init__(self, cfgs, tables=(), stream=None, torch_alloc=True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the PIC library runs only on an MI355X")
        L = load_library()
        if isinstance(cfgs, dict):
            cfgs = [cfgs]
        self.cfgs = list(cfgs)
        self.B = len(self.cfgs)
        self.S = len(self.cfgs[0]["species"])
        arr = (PicConfig * self.B)(*[make_config(c) for c in self.cfgs])
        self._torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._alloc = None
        if torch_alloc:
            dev = torch.cuda.current_device()
            strm = self.stream

            def _a(nbytes, user):
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, strm)

            def _f(ptr, user):
                if torch.cuda is not None:
                    torch.cuda.caching_allocator_delete(ptr)

            self._afn, self._ffn = ALLOC_FN(_a), FREE_FN(_f)
            self._alloc = PicAllocator(self._afn, self._ffn, None)
        h = C.c_void_p()
        rc = L.pic_init(arr, self.B, C.byref(self._alloc) if self._alloc else None,
                        C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != OK:
            raise PicError(rc, "pic_init")
        self.h = h
        _live.append(weakref.ref(self))
        self.n_nodes = [c["n_cells"] + (1 if c["bc"] == 1 else 0) for c in self.cfgs]
        self.tables = []            # every table loaded, in order (checkpoints replay them)
        self.retired = set()
        for t in tables:
            self.load_xsec(t["species"], t["kind"], t["threshold"], t["energy"], t["sigma"],
                           batch=t.get("batch", -1))

    def close(self):
        if getattr(self, "h", None):
            _lib.pic_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != OK:
            raise PicError(rc, what)

    def load_xsec(self, species, kind, threshold, energy, sigma, batch=-1):
        e = np.ascontiguousarray(energy, dtype=np.float64)
        s = np.ascontiguousarray(sigma, dtype=np.float64)
        self._check(_lib.pic_load_xsec(self.h, batch, species, kind, threshold, len(e),
                                       _ptr(e, C.c_double), _ptr(s, C.c_double)), "pic_load_xsec")
        self.tables.append(dict(species=int(species), kind=int(kind), threshold=float(threshold),
                                energy=e.copy(), sigma=s.copy(), batch=int(batch)))

    def step(self, n=1):
        self._check(_lib.pic_step(self.h, int(n)), "pic_step")

    def sync(self, check=True):
        rc = _lib.pic_sync(self.h)
        if check:
            self._check(rc, "pic_sync")

    def config_tiles(self, ppt=4, threads=256, sort_every=0, compact_every=16):
        self._check(_lib.pic_config_tiles(self.h, ppt, threads, sort_every, compact_every), "pic_config_tiles")

    def thin(self, species, above, keep):
        """In every running discharge whose `species` holds more than `above`
        particles, keep each with probability keep / live (on the device; the
        survivors keep their order and ids)."""
        self._check(_lib.pic_thin(self.h, int(species), int(above), int(keep)), "pic_thin")

    def config_events(self, in_push=False):
        """Events (collisions, renewals, secondary emission) in the push
        workgroups of a 256-thread tile (True) or in the events kernel."""
        self._check(_lib.pic_config_events(self.h, int(bool(in_push))), "pic_config_events")

    def set_diag(self, enable=True, eepf_emax=64.0):
        self._check(_lib.pic_set_diag(self.h, int(enable), float(eepf_emax)), "pic_set_diag")

    def set_wall_edf(self, species, emax):
        """Energy range [0, emax) eV of species' wall impact-energy histograms."""
        self._check(_lib.pic_set_wall_edf(self.h, int(species), float(emax)), "pic_set_wall_edf")

    def poisson(self, t, rho=None, batch=0):
        n = self.n_nodes[batch]
        phi, ef = np.zeros(n), np.zeros(n)
        r = None
        if rho is not None:
            r = np.ascontiguousarray(rho, dtype=np.float64)
            assert r.shape == (n,)
        self._check(_lib.pic_poisson(self.h, batch, float(t),
                                     _ptr(r, C.c_double) if r is not None else None,
                                     _ptr(phi, C.c_double), _ptr(ef, C.c_double)), "pic_poisson")
        return phi, ef

    def diag(self, what, count, dtype=np.float64, batch=0, check=True):
        out = np.zeros(count, dtype=dtype)
        rc = _lib.pic_diag(self.h, batch, DIAG[what], out.ctypes.data_as(C.c_void_p), out.nbytes)
        if check:
            self._check(rc, f"pic_diag({what})")
        return out

    def counts(self, batch=0):
        o = self.diag("COUNTS", 4 + 2 * self.S, np.int64, batch, check=False)
        return dict(step=int(o[0]), n_nodes=int(o[1]), flags=int(o[3]),
                    count=[int(o[4 + 2 * s]) for s in range(self.S)],
                    next_id=[int(o[5 + 2 * s]) for s in range(self.S)])

    def rho(self, batch=0):
        return self.diag("RHO", self.n_nodes[batch], batch=batch)

    def phi(self, batch=0):
        return self.diag("PHI", self.n_nodes[batch], batch=batch)

    def efield(self, batch=0):
        return self.diag("EFIELD", self.n_nodes[batch], batch=batch)

    def density(self, batch=0):
        n = self.n_nodes[batch]
        return self.diag("DENSITY", self.S * n, batch=batch).reshape(self.S, n)

    def energy(self, batch=0):
        o = self.diag("ENERGY", self.S + 1, batch=batch)
        return o[: self.S].copy(), float(o[self.S])

    def wall(self, batch=0):
        o = self.diag("WALL", 2 * self.S + 2, np.int64, batch)
        return dict(absorbed=o[: 2 * self.S].reshape(self.S, 2), see_emitted=o[2 * self.S:])

    def coll(self, batch=0):
        o = self.diag("COLL", self.S * (3 + MAX_CHAN), np.int64, batch).reshape(self.S, 3 + MAX_CHAN)
        return dict(candidates=o[:, 0], nulls=o[:, 1], violations=o[:, 2], coll=o[:, 3:])

    def numax(self, species, batch=0):
        o = self.diag("NUMAX", 2 * self.S, batch=batch)
        return float(o[species]), int(o[self.S + species])

    def flags(self, batch=0):
        return int(self.diag("FLAGS", 1, np.int64, batch)[0])

    def avg(self, batch=0, check=True):
        n = self.n_nodes[batch]
        o = self.diag("AVG", 1 + (self.S + 2) * n, batch=batch, check=check)
        prof = o[1:].reshape(self.S + 2, n)
        return dict(samples=o[0], density=prof[: self.S], phi=prof[self.S], mean_energy=prof[self.S + 1])

    def wall_energy(self, batch=0):
        """Kinetic energy carried into each wall per species since start, J/m^2,
        as [S][2] (wall at x < 0, wall at x >= L)."""
        return self.diag("WALL_ENERGY", 2 * self.S, batch=batch).reshape(self.S, 2)

    def power(self, batch=0):
        """Time means per species: flux density, x-momentum flux density, the
        power density q Gamma E the field gives the species and its
        decomposition into inertia, pressure and the ohmic rest."""
        n = self.n_nodes[batch]
        o = self.diag("POWER", 1 + 5 * self.S * n, batch=batch)
        p = o[1:].reshape(self.S, 5, n)
        return dict(samples=o[0], flux=p[:, 0], momentum=p[:, 1], power=p[:, 2], inertia=p[:, 3],
                    pressure=p[:, 4], ohmic=p[:, 2] - p[:, 3] - p[:, 4])

    def eepf(self, batch=0):
        o = self.diag("EEPF", 2 * EEPF_BINS + 2, batch=batch)
        return dict(bulk=o[:EEPF_BINS], wall=o[EEPF_BINS:2 * EEPF_BINS],
                    bin_width=o[2 * EEPF_BINS], samples=o[2 * EEPF_BINS + 1])

    def wall_edf(self, batch=0):
        """Impact-energy histograms [species][wall][bin] since the last reset
        (wall 0 at x < 0, wall 1 at x >= L), bin width per species (eV), and
        the samples of the time averages over the same interval."""
        S = self.S
        nv = S * 2 * EEPF_BINS
        o = self.diag("WALL_EDF", nv + S + 1, batch=batch)
        return dict(counts=o[:nv].reshape(S, 2, EEPF_BINS), bin_width=o[nv:nv + S], samples=o[nv + S])

    def reset_avg(self, batch=0, check=True):
        rc = _lib.pic_diag(self.h, batch, DIAG["RESET_AVG"], None, 0)
        if check:
            self._check(rc, "pic_diag(RESET_AVG)")

    def load_profiles(self, density, temp_ev, n, batch=0):
        """Restart discharge `batch` from profiles [S][m] (relative density,
        temperature in eV) with n[s] particles of species s."""
        dens = np.ascontiguousarray(density, dtype=np.float64)
        temp = np.ascontiguousarray(temp_ev, dtype=np.float64)
        if dens.shape != temp.shape or dens.shape[0] != self.S:
            raise ValueError("density and temperature must both be [n_species, m]")
        nn = (C.c_int64 * self.S)(*[int(v) for v in n])
        self._check(_lib.pic_load_profiles(self.h, batch, dens.shape[1], _ptr(dens, C.c_double),
                                           _ptr(temp, C.c_double), nn), "pic_load_profiles")

    def retire(self, batch, retired=True):
        self._check(_lib.pic_retire(self.h, batch, int(retired)), "pic_retire")
        if retired:
            self.retired.add(int(batch))
        else:
            self.retired.discard(int(batch))

    def sort(self):
        self._check(_lib.pic_sort(self.h), "pic_sort")

    def sort_noalloc(self):
        """pic_sort with the library's fixed per-GPU scratch: no allocation."""
        self._check(_lib.pic_sort_noalloc(self.h), "pic_sort_noalloc")

    def use_graphs(self, enable=True):
        self._check(_lib.pic_use_graphs(self.h, int(enable)), "pic_use_graphs")

    def profile(self, enable=True):
        self._check(_lib.pic_profile(self.h, int(enable)), "pic_profile")

    def graphs(self):
        """Replays of captured step graphs since the start, and the steps they ran."""
        o = self.diag("GRAPHS", 2, np.int64)
        return dict(replays=int(o[0]), steps=int(o[1]))

    def timing(self):
        o = self.diag("TIMING", 6)
        return dict(finalize_n=float(o[0]), finalize_ms=float(o[1]),
                    push_n=float(o[2]), push_ms=float(o[3]),
                    events_n=float(o[4]), events_ms=float(o[5]))

    def charge(self, batch=0):
        o = self.diag("CHARGE", 2, batch=batch)
        return float(o[0]), float(o[1])

    def get_particles(self, species, batch=0):
        n = C.c_int64()
        nid = C.c_uint32()
        self._check(_lib.pic_get_particles(self.h, batch, species, 0, None, None, None, None, None,
                                           None, C.byref(n), C.byref(nid)), "pic_get_particles")
        m = n.value
        cell = np.zeros(m, np.int32)
        off, vx, vy, vz = (np.zeros(m, np.float32) for _ in range(4))
        ids = np.zeros(m, np.uint32)
        self._check(_lib.pic_get_particles(self.h, batch, species, m, _ptr(cell, C.c_int32),
                                           _ptr(off, C.c_float), _ptr(vx, C.c_float),
                                           _ptr(vy, C.c_float), _ptr(vz, C.c_float),
                                           _ptr(ids, C.c_uint32), C.byref(n), C.byref(nid)),
                    "pic_get_particles")
        return dict(cell=cell, off=off, vx=vx, vy=vy, vz=vz, id=ids, next_id=nid.value)

    def circuit(self, batch=0):
        """(potential of the electrode at x = 0 at the last solve, charge per
        area of its conductor; 0 without a circuit)."""
        o = self.diag("CIRCUIT", 2, batch=batch)
        return float(o[0]), float(o[1])

    def set_circuit(self, q, batch=0):
        self._check(_lib.pic_set_circuit(self.h, batch, float(q)), "pic_set_circuit")

    def set_windows(self, batch, steps):
        """Close an averaging window of discharge `batch` every `steps` steps
        on the device (0: off)."""
        self._check(_lib.pic_set_windows(self.h, batch, int(steps)), "pic_set_windows")

    def windows(self, batch=0, first=0, count=None):
        """Completed windows first .. (all completed when count is None), each
        a dict as avg()."""
        n = C.c_int64()
        self._check(_lib.pic_get_windows(self.h, batch, first, 0, None, C.byref(n)), "pic_get_windows")
        cnt = n.value - first if count is None else count
        if cnt <= 0:
            return []
        nn = self.n_nodes[batch]
        row = 1 + (self.S + 2) * nn
        o = np.zeros(cnt * row)
        self._check(_lib.pic_get_windows(self.h, batch, first, cnt, _ptr(o, C.c_double), C.byref(n)),
                    "pic_get_windows")
        out = []
        for k in range(cnt):
            r = o[k * row:(k + 1) * row]
            prof = r[1:].reshape(self.S + 2, nn)
            out.append(dict(samples=r[0], density=prof[: self.S], phi=prof[self.S], mean_energy=prof[self.S + 1]))
        return out

    def renewed(self, batch=0):
        """Axial renewals per species since the start."""
        return self.diag("RENEWED", self.S, np.int64, batch).copy()

    def axial(self, species, batch=0):
        """Axial displacements (m) of a species, in the order of get_particles
        (renewal only)."""
        n = C.c_int64()
        self._check(_lib.pic_get_axial(self.h, batch, species, 0, None, C.byref(n)), "pic_get_axial")
        z = np.zeros(n.value, np.float64)
        self._check(_lib.pic_get_axial(self.h, batch, species, n.value, _ptr(z, C.c_double), C.byref(n)),
                    "pic_get_axial")
        return z

    def set_axial(self, species, z, batch=0):
        z = np.ascontiguousarray(z, np.float64)
        self._check(_lib.pic_set_axial(self.h, batch, species, len(z), _ptr(z, C.c_double)), "pic_set_axial")

    def set_particles(self, species, cell, off, vx, vy, vz, ids, next_id, step, batch=0):
        cell = np.ascontiguousarray(cell, np.int32)
        off, vx, vy, vz = (np.ascontiguousarray(a, np.float32) for a in (off, vx, vy, vz))
        ids = np.ascontiguousarray(ids, np.uint32)
        self._check(_lib.pic_set_particles(self.h, batch, species, len(cell), _ptr(cell, C.c_int32),
                                           _ptr(off, C.c_float), _ptr(vx, C.c_float),
                                           _ptr(vy, C.c_float), _ptr(vz, C.c_float),
                                           _ptr(ids, C.c_uint32), int(next_id), int(step)),
                    "pic_set_particles")


def declared_functions(headers=None):
    """Names of the functions the headers under ``include/`` declare."""
    import re
    inc = os.path.join(os.path.dirname(HERE), "include")
    headers = headers or [os.path.join(inc, h) for h in ("pic.h", "pic_mlp.h")]
    names = set()
    for h in headers:
        names |= set(re.findall(r"\b(pic_[a-z_]+)\s*\(", open(h).read()))
    return sorted(names)


class MLP:
    """The warm-start network (``pic_mlp``): BF16 matrix-core training and
    inference; inputs, targets and outputs are float32 CUDA tensors."""

    def __init__(self, widths, max_batch, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the network runs only on an MI355X")
        L = load_library()
        self._torch = torch
        self.widths = tuple(int(w) for w in widths)
        self.max_batch = int(max_batch)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        w = (C.c_int32 * len(self.widths))(*self.widths)
        h = C.c_void_p()
        rc = L.pic_mlp_create(w, len(self.widths), self.max_batch, None, C.c_void_p(self.stream.cuda_stream),
                              C.byref(h))
        if rc != OK:
            raise PicError(rc, "pic_mlp_create")
        self.h = h
        self.n_params = int(L.pic_mlp_n_params(h))
        self._loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        _live.append(weakref.ref(self))

    def close(self):
        if getattr(self, "h", None):
            _lib.pic_mlp_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != OK:
            raise PicError(rc, what)

    def _dev(self, a, cols):
        t = self._torch
        a = t.as_tensor(a, dtype=t.float32, device="cuda").contiguous()
        if a.dim() != 2 or a.shape[1] != cols:
            raise ValueError(f"expected [batch, {cols}], got {tuple(a.shape)}")
        return a

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        self._check(_lib.pic_mlp_set_params(self.h, _ptr(p, C.c_float), p.size), "pic_mlp_set_params")

    def params(self):
        p = np.empty(self.n_params, dtype=np.float32)
        self._check(_lib.pic_mlp_get_params(self.h, _ptr(p, C.c_float), p.size), "pic_mlp_get_params")
        return p

    def forward(self, x):
        x = self._dev(x, self.widths[0])
        y = self._torch.empty((x.shape[0], self.widths[-1]), dtype=self._torch.float32, device="cuda")
        self._check(_lib.pic_mlp_forward(self.h, x.shape[0], x.data_ptr(), y.data_ptr()), "pic_mlp_forward")
        self._keep = x
        return y

    def train_step(self, x, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, loss_out=None):
        """One Adam update; returns the batch loss as a 1-element CUDA tensor
        (taken before the update; written into `loss_out` when given)."""
        x, t = self._dev(x, self.widths[0]), self._dev(t, self.widths[-1])
        loss = loss_out if loss_out is not None else self._torch.empty(1, dtype=self._torch.float32, device="cuda")
        self._check(_lib.pic_mlp_train_step(self.h, x.shape[0], x.data_ptr(), t.data_ptr(), lr, beta1, beta2,
                                            eps, loss.data_ptr()), "pic_mlp_train_step")
        self._keep = (x, t)
        return loss

    def grad(self, x, t):
        x, t = self._dev(x, self.widths[0]), self._dev(t, self.widths[-1])
        g = np.empty(self.n_params, dtype=np.float32)
        loss = np.empty(1, dtype=np.float32)
        self._check(_lib.pic_mlp_grad(self.h, x.shape[0], x.data_ptr(), t.data_ptr(), _ptr(g, C.c_float),
                                      _ptr(loss, C.c_float)), "pic_mlp_grad")
        return float(loss[0]), g

    def sync(self):
        self._check(_lib.pic_mlp_sync(self.h), "pic_mlp_sync")
