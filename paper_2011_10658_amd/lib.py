"""ctypes binding of libqedttn (argument marshalling only).

Names follow the C ABI in include/qedttn.h with the `qed_` prefix dropped.
Device buffers are passed as raw pointers (e.g. torch CUDA tensors'
data_ptr()); PyTorch is only used by callers for memory and streams.
Every call checks the status code and raises QedError on failure.
"""

import ctypes as C
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# QEDTTN_LIBRARY names another build of the same library (the host-sanitizer
# build used by the CPU tests); the in-tree build otherwise
LIBPATH = os.environ.get("QEDTTN_LIBRARY") or os.path.join(HERE, "libqedttn.so")

OK, NOT_CONVERGED = 0, 1
ERR = {-1: "INVALID_ARG", -2: "BAD_STATE", -3: "OOM", -4: "HIP", -6: "NONFINITE",
       -7: "UNSUPPORTED", -8: "IO"}
BC_OPEN_ZERO_FLUX, BC_OPEN_FREE_FLUX, BC_PERIODIC = 0, 1, 2
FP64, FP32, BF16 = 0, 1, 2


class QedError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERR.get(code, code)}: {msg}")
        self.code = code


class SweepReport(C.Structure):
    _fields_ = [("energy", C.c_double), ("dE", C.c_double), ("nu", C.c_double),
                ("deltaL", C.c_double), ("Q", C.c_double), ("seconds", C.c_double),
                ("flops", C.c_double), ("matvecs", C.c_longlong)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Stats(C.Structure):
    _fields_ = [("matvec_flops", C.c_double), ("matvecs", C.c_longlong),
                ("gemm_launches", C.c_longlong), ("gemm_ms", C.c_double),
                ("gemm_flops", C.c_double), ("fused_launches", C.c_longlong),
                ("fused_ms", C.c_double), ("fused_flops", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Term(C.Structure):
    _fields_ = [("coef", C.c_double), ("op", C.c_void_p * 3), ("shift", C.c_int * 3)]


class HeffDesc(C.Structure):
    _fields_ = [("ch", C.POINTER(C.c_int) * 3), ("n", C.POINTER(C.c_int) * 3),
                ("nsec", C.c_int * 3), ("K", C.c_int), ("terms", C.POINTER(Term))]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)

_lib = None

_P = C.c_void_p
_I = C.c_int
_D = C.c_double
_IP = C.POINTER(C.c_int)
_DP = C.POINTER(C.c_double)
_LP = C.POINTER(C.c_int64)

SIGNATURES = {
    "qed_create": [C.POINTER(_P), _I],
    "qed_destroy": [_P],
    "qed_last_error": [_P],
    "qed_set_allocator": [_P, ALLOC_FN, FREE_FN, _P],
    "qed_set_stream": [_P, _P],
    "qed_set_lattice": [_P, _I, _I, _I, _I],
    "qed_set_couplings": [_P, _D, _D, _D, _D],
    "qed_set_chemical_potential": [_P, _DP],
    "qed_physical_line": [_D, _D, _DP, _DP],
    "qed_set_penalty": [_P, _D, _I, _I, _I],
    "qed_set_charge_sector": [_P, _I],
    "qed_set_bond_dim": [_P, _I],
    "qed_set_lanczos": [_P, _I, _I, _D],
    "qed_set_lanczos_schedule": [_P, C.c_double, C.c_double],
    "qed_set_precision": [_P, _I, _I],
    "qed_build_hamiltonian": [_P],
    "qed_get_local_dims": [_P, _IP],
    "qed_get_tree": [_P, _IP, _IP],
    "qed_get_node_links": [_P, _I, _IP],
    "qed_get_leg_sectors": [_P, _I, _IP, _IP, _I, _IP],
    "qed_init_state": [_P, C.c_uint64],
    "qed_set_node": [_P, _I, _DP, C.c_int64],
    "qed_get_node": [_P, _I, _DP, C.c_int64],
    "qed_node_size": [_P, _I, _LP],
    "qed_sweep": [_P, _I, C.POINTER(SweepReport)],
    "qed_save_state": [_P, C.c_char_p],
    "qed_load_state": [_P, C.c_char_p],
    "qed_debug_poison": [_P, _I],
    "qed_get_energy": [_P, _DP],
    "qed_get_observables": [_P, _DP, _DP, _DP, _DP, _DP],
    "qed_get_site_fluxes": [_P, _DP, _DP],
    "qed_set_expansion": [_P, C.c_int, C.c_double, C.c_int, C.c_int, C.c_uint64],
    "qed_get_plane_profiles": [_P, C.c_int, _DP, _DP],
    "qed_get_surface_density": [_P, _DP, _IP],
    "qed_pin_charges": [_P, C.c_int, _IP, _IP, C.c_double],
    "qed_heff_batch_create": [_P, _I, C.POINTER(HeffDesc), C.POINTER(_P)],
    "qed_heff_batch_destroy": [_P],
    "qed_heff_batch_size": [_P, _LP, _LP],
    "qed_heff_batch_matvec": [_P, _P, _P],
    "qed_heff_batch_lanczos": [_P, _P, _I, _DP, _DP, _I],
    "qed_heff_batch_flops": [_P, _DP, _DP],
    "qed_autotune": [_P, C.c_char_p],
    "qed_set_profiling": [_P, _I],
    "qed_get_stats": [_P, C.POINTER(Stats)],
    "qed_node_blocks": [_IP, _IP, _I, _IP, _IP, _I, _IP, _IP, _I, _I, _I, _IP, _IP, _LP],
    "qed_heff_create": [_P, _IP, _IP, _I, _IP, _IP, _I, _IP, _IP, _I, _I,
                        C.POINTER(Term), C.POINTER(_P)],
    "qed_heff_destroy": [_P],
    "qed_heff_size": [_P, _LP],
    "qed_heff_matvec": [_P, _P, _P],
    "qed_heff_matvec_noalloc": [_P, _P, _P],
    "qed_heff_lanczos": [_P, _P, _I, _DP, _DP],
    "qed_heff_flops": [_P, _DP, _DP],
    "qed_heff_matvec_adjoint": [_P, _P, _P, _P, C.POINTER(_P), _DP],
    "qed_heff_adjoint_flops": [_P, _DP, _DP],
}


def load():
    """Load the in-tree library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise ImportError(
            f"{LIBPATH} is missing: build it with `python -m paper_2011_10658_amd.build`")
    lib = C.CDLL(LIBPATH)
    for name, args in SIGNATURES.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_char_p if name == "qed_last_error" else C.c_int
    _lib = lib
    return lib


def _ia(seq):
    a = (C.c_int * max(1, len(seq)))(*seq)
    return a


def _check(rc, ctx=None, ok=(OK,)):
    if rc in ok:
        return rc
    msg = ""
    if ctx is not None:
        m = load().qed_last_error(ctx)
        msg = m.decode() if m else ""
    raise QedError(rc, msg)


def physical_line(g2, t=1.0):
    a, b = C.c_double(), C.c_double()
    _check(load().qed_physical_line(g2, t, C.byref(a), C.byref(b)))
    return a.value, b.value


def node_blocks(l, r, p, flux=0):
    """Block table of a three-leg tensor: legs as [(q, n)].  Returns
    (triples [(il, ir, ip)], offsets np.int64[nblk+1])."""
    lib = load()
    args = []
    for leg in (l, r, p):
        args += [_ia([q for q, _ in leg]), _ia([n for _, n in leg]), len(leg)]
    nblk = C.c_int()
    _check(lib.qed_node_blocks(*args, flux, 0, C.byref(nblk), None, None))
    nb = nblk.value
    tr = (C.c_int * max(1, 3 * nb))()
    offs = (C.c_int64 * (nb + 1))()
    _check(lib.qed_node_blocks(*args, flux, nb, C.byref(nblk), tr, offs))
    triples = [(tr[3 * b], tr[3 * b + 1], tr[3 * b + 2]) for b in range(nb)]
    return triples, np.array(offs[:], dtype=np.int64)


class Context:
    """One library context.  device=-1 gives a host-only context."""

    def __init__(self, device=0):
        self.lib = load()
        h = C.c_void_p()
        _check(self.lib.qed_create(C.byref(h), device))
        self.h = h
        self._keep = []
        self._children = weakref.WeakSet()

    def close(self):
        """Destroy the context; H_eff objects made from it are closed
        first (they use its device allocator and stream)."""
        for child in list(self._children):
            child.close()
        if self.h:
            self.lib.qed_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _c(self, rc, ok=(OK,)):
        return _check(rc, self.h, ok)

    def set_stream(self, stream_ptr):
        self._c(self.lib.qed_set_stream(self.h, C.c_void_p(stream_ptr)))

    def set_allocator(self, alloc, free):
        """alloc(bytes, stream) -> int pointer; free(ptr, stream)."""
        a = ALLOC_FN(lambda n, s, u: alloc(int(n), s))
        f = FREE_FN(lambda p, s, u: free(p, s))
        self._keep += [a, f]
        self._c(self.lib.qed_set_allocator(self.h, a, f, None))

    def set_lattice(self, Lx, Ly, Lz, bc=BC_OPEN_ZERO_FLUX):
        self._c(self.lib.qed_set_lattice(self.h, Lx, Ly, Lz, bc))
        self._nsites = Lx * Ly * Lz
        self._dims = (Lx, Ly, Lz)

    def set_couplings(self, t, m, g2e, g2m):
        self._c(self.lib.qed_set_couplings(self.h, t, m, g2e, g2m))

    def set_chemical_potential(self, mu):
        """mu: one value per site (site order), or None to remove."""
        if mu is None:
            self._c(self.lib.qed_set_chemical_potential(self.h, None))
            return
        a = np.ascontiguousarray(mu, dtype=np.float64).reshape(-1)
        if a.size != getattr(self, "_nsites", -1):
            raise ValueError("need one chemical potential per site (call set_lattice first)")
        self._c(self.lib.qed_set_chemical_potential(self.h, a.ctypes.data_as(_DP)))

    def set_penalty(self, nu_max, n_linear=0, n_quadratic=0, adaptive=0):
        self._c(self.lib.qed_set_penalty(self.h, nu_max, n_linear, n_quadratic, adaptive))

    def set_charge_sector(self, Q):
        self._c(self.lib.qed_set_charge_sector(self.h, Q))

    def set_bond_dim(self, chi):
        self._c(self.lib.qed_set_bond_dim(self.h, chi))

    def set_lanczos(self, steps, cycles=1, tol=0.0):
        self._c(self.lib.qed_set_lanczos(self.h, steps, cycles, tol))

    def set_expansion(self, alpha, delta, chi_max=0, seed=0, on=True):
        """Subspace expansion (SVD moves; links grow by up to delta columns
        per sector on the move after an update); on=False switches it off."""
        self._c(self.lib.qed_set_expansion(self.h, 1 if on else 0, alpha, delta, chi_max, seed))

    def set_lanczos_schedule(self, tol0, factor=0.1):
        self._c(self.lib.qed_set_lanczos_schedule(self.h, tol0, factor))

    def set_precision(self, dtype, refine=1):
        self._c(self.lib.qed_set_precision(self.h, dtype, refine))

    def build_hamiltonian(self):
        self._c(self.lib.qed_build_hamiltonian(self.h))

    def tree(self):
        nn, ns = C.c_int(), C.c_int()
        self._c(self.lib.qed_get_tree(self.h, C.byref(nn), C.byref(ns)))
        return nn.value, ns.value

    def local_dims(self):
        _, ns = self.tree()
        d = (C.c_int * ns)()
        self._c(self.lib.qed_get_local_dims(self.h, d))
        return list(d)

    def node_links(self, node):
        a = (C.c_int * 3)()
        self._c(self.lib.qed_get_node_links(self.h, node, a))
        return tuple(a)

    def leg_sectors(self, link):
        n = C.c_int()
        self._c(self.lib.qed_get_leg_sectors(self.h, link, None, None, 0, C.byref(n)))
        q = (C.c_int * max(1, n.value))()
        s = (C.c_int * max(1, n.value))()
        self._c(self.lib.qed_get_leg_sectors(self.h, link, q, s, n.value, C.byref(n)))
        return [(q[i], s[i]) for i in range(n.value)]

    def init_state(self, seed):
        self._c(self.lib.qed_init_state(self.h, C.c_uint64(seed)))

    def node_size(self, node):
        n = C.c_int64()
        self._c(self.lib.qed_node_size(self.h, node, C.byref(n)))
        return n.value

    def set_node(self, node, flat):
        a = np.ascontiguousarray(flat, dtype=np.float64)
        self._c(self.lib.qed_set_node(self.h, node, a.ctypes.data_as(_DP), a.size))

    def get_node(self, node):
        a = np.zeros(self.node_size(node))
        self._c(self.lib.qed_get_node(self.h, node, a.ctypes.data_as(_DP), a.size))
        return a

    def sweep(self, n=1, report=True):
        """Run n sweeps; with report=True each sweep also measures the
        local observables (delta_L, Q) for its record."""
        if not report:
            self._c(self.lib.qed_sweep(self.h, n, None))
            return None
        reps = (SweepReport * max(1, n))()
        self._c(self.lib.qed_sweep(self.h, n, reps))
        return [reps[i].as_dict() for i in range(n)]

    def save_state(self, path):
        self._c(self.lib.qed_save_state(self.h, os.fsencode(path)))

    def load_state(self, path):
        self._c(self.lib.qed_load_state(self.h, os.fsencode(path)))

    def debug_poison(self, node):
        self._c(self.lib.qed_debug_poison(self.h, node))

    def energy(self):
        e = C.c_double()
        self._c(self.lib.qed_get_energy(self.h, C.byref(e)))
        return e.value

    def observables(self):
        _, ns = self.tree()
        occ = np.zeros(ns)
        ef = np.zeros(3 * ns)
        dL, rho, Q = C.c_double(), C.c_double(), C.c_double()
        self._c(self.lib.qed_get_observables(self.h, occ.ctypes.data_as(_DP),
                                             ef.ctypes.data_as(_DP), C.byref(dL),
                                             C.byref(rho), C.byref(Q)))
        return dict(occ=occ, efield=ef.reshape(ns, 3), deltaL=dL.value, rho=rho.value,
                    Q=Q.value)

    def site_fluxes(self):
        """(charge[N], flux[N, 6]): Gauss-law charge and outgoing half-link
        fluxes per site."""
        ns = self._nsites
        q, f = np.zeros(ns), np.zeros(6 * ns)
        self._c(self.lib.qed_get_site_fluxes(self.h, q.ctypes.data_as(_DP), f.ctypes.data_as(_DP)))
        return q, f.reshape(ns, 6)

    def plane_profiles(self, axis):
        """(qc[L_a], ec[L_a + 1]) along `axis`."""
        if axis not in (0, 1, 2):
            raise ValueError("axis must be 0, 1 or 2")
        La = self._dims[axis]
        qc, ec = np.zeros(La), np.zeros(La + 1)
        self._c(self.lib.qed_get_plane_profiles(self.h, axis, qc.ctypes.data_as(_DP),
                                                ec.ctypes.data_as(_DP)))
        return qc, ec

    def surface_density(self):
        n = C.c_int()
        self._c(self.lib.qed_get_surface_density(self.h, None, C.byref(n)))
        sig = np.zeros(n.value)
        self._c(self.lib.qed_get_surface_density(self.h, sig.ctypes.data_as(_DP), C.byref(n)))
        return sig

    def pin_charges(self, pins, lam):
        """pins: {site: charge in (-1, 0, +1)}; adds pinning potentials."""
        sites = np.ascontiguousarray(list(pins.keys()), dtype=np.int32)
        qs = np.ascontiguousarray(list(pins.values()), dtype=np.int32)
        self._c(self.lib.qed_pin_charges(self.h, len(sites), sites.ctypes.data_as(_IP),
                                         qs.ctypes.data_as(_IP), lam))

    def set_profiling(self, on):
        self._c(self.lib.qed_set_profiling(self.h, 1 if on else 0))

    def stats(self):
        st = Stats()
        self._c(self.lib.qed_get_stats(self.h, C.byref(st)))
        return st.as_dict()

    def autotune(self, cache_path=None):
        """Enable the tile-shape autotuner (None: in-memory cache only;
        "": disable)."""
        arg = None if cache_path is None else cache_path.encode()
        self._c(self.lib.qed_autotune(self.h, arg))

    def heff_batch(self, nodes):
        """nodes: [((l, r, p), terms)] with terms as in heff()."""
        return HeffBatch(self, nodes)

    def heff(self, l, r, p, terms):
        """terms: [(coef, (ptr_l, ptr_r, ptr_p), (shift_l, shift_r, shift_p))]
        with device FP64 operator pointers (0 / None = identity)."""
        return Heff(self, l, r, p, terms)


class Heff:
    def __init__(self, ctx, l, r, p, terms):
        self.ctx = ctx
        lib = ctx.lib
        args = []
        for leg in (l, r, p):
            args += [_ia([q for q, _ in leg]), _ia([n for _, n in leg]), len(leg)]
        arr = (Term * max(1, len(terms)))()
        for k, (c, ptrs, shifts) in enumerate(terms):
            arr[k].coef = c
            for e in range(3):
                arr[k].op[e] = ptrs[e] or None
                arr[k].shift[e] = shifts[e]
        h = C.c_void_p()
        ctx._c(lib.qed_heff_create(ctx.h, *args, len(terms), arr, C.byref(h)))
        self.h = h
        ctx._children.add(self)
        n = C.c_int64()
        _check(lib.qed_heff_size(h, C.byref(n)))
        self.size = n.value

    def close(self):
        if self.h and self.ctx.h:
            self.ctx.lib.qed_heff_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def matvec(self, x_ptr, y_ptr):
        self.ctx._c(self.ctx.lib.qed_heff_matvec(self.h, C.c_void_p(x_ptr), C.c_void_p(y_ptr)))

    def matvec_noalloc(self, x_ptr, y_ptr):
        self.ctx._c(self.ctx.lib.qed_heff_matvec_noalloc(self.h, C.c_void_p(x_ptr),
                                                         C.c_void_p(y_ptr)))

    def lanczos(self, x_ptr, steps=0):
        ev, res = C.c_double(), C.c_double()
        rc = self.ctx._c(self.ctx.lib.qed_heff_lanczos(self.h, C.c_void_p(x_ptr), steps,
                                                       C.byref(ev), C.byref(res)),
                         ok=(OK, NOT_CONVERGED))
        return ev.value, res.value, rc

    def flops(self):
        f, b = C.c_double(), C.c_double()
        _check(self.ctx.lib.qed_heff_flops(self.h, C.byref(f), C.byref(b)))
        return f.value, b.value

    def adjoint_flops(self):
        a, b = C.c_double(), C.c_double()
        self.ctx._c(self.ctx.lib.qed_heff_adjoint_flops(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def adjoint(self, x_ptr, ybar_ptr, xbar_ptr=0, opbar_ptrs=None, want_coefbar=False, K=None):
        """Reverse mode of y = H_eff x.  opbar_ptrs: list of 3K device
        pointers (0 = skip).  Returns coefbar (np array) or None."""
        ob = None
        if opbar_ptrs is not None:
            ob = (C.c_void_p * len(opbar_ptrs))(*[p or None for p in opbar_ptrs])
        cb = np.zeros(K) if want_coefbar else None
        self.ctx._c(self.ctx.lib.qed_heff_matvec_adjoint(
            self.h, C.c_void_p(x_ptr), C.c_void_p(ybar_ptr), C.c_void_p(xbar_ptr or None), ob,
            cb.ctypes.data_as(_DP) if cb is not None else None))
        return cb


class HeffBatch:
    def __init__(self, ctx, nodes):
        self.ctx = ctx
        lib = ctx.lib
        self._keep = []
        descs = (HeffDesc * len(nodes))()
        for i, (legs, terms) in enumerate(nodes):
            for e in range(3):
                q = _ia([c for c, _ in legs[e]])
                n = _ia([s for _, s in legs[e]])
                self._keep += [q, n]
                descs[i].ch[e] = C.cast(q, C.POINTER(C.c_int))
                descs[i].n[e] = C.cast(n, C.POINTER(C.c_int))
                descs[i].nsec[e] = len(legs[e])
            arr = (Term * max(1, len(terms)))()
            for k, (c, ptrs, shifts) in enumerate(terms):
                arr[k].coef = c
                for e in range(3):
                    arr[k].op[e] = ptrs[e] or None
                    arr[k].shift[e] = shifts[e]
            self._keep.append(arr)
            descs[i].K = len(terms)
            descs[i].terms = C.cast(arr, C.POINTER(Term))
        h = C.c_void_p()
        ctx._c(lib.qed_heff_batch_create(ctx.h, len(nodes), descs, C.byref(h)))
        self.h = h
        self.nn = len(nodes)
        ctx._children.add(self)
        tot = C.c_int64()
        offs = (C.c_int64 * (self.nn + 1))()
        _check(lib.qed_heff_batch_size(h, C.byref(tot), offs))
        self.size = tot.value
        self.offsets = np.array(offs[:], dtype=np.int64)

    def close(self):
        if self.h and self.ctx.h:
            self.ctx.lib.qed_heff_batch_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def matvec(self, x_ptr, y_ptr):
        self.ctx._c(self.ctx.lib.qed_heff_batch_matvec(self.h, C.c_void_p(x_ptr), C.c_void_p(y_ptr)))

    def lanczos(self, x_ptr, steps=0, graph=True):
        ev = np.zeros(self.nn)
        res = np.zeros(self.nn)
        rc = self.ctx._c(self.ctx.lib.qed_heff_batch_lanczos(
            self.h, C.c_void_p(x_ptr), steps, ev.ctypes.data_as(_DP), res.ctypes.data_as(_DP),
            1 if graph else 0), ok=(OK, NOT_CONVERGED))
        return ev, res, rc

    def flops(self):
        f, b = C.c_double(), C.c_double()
        _check(self.ctx.lib.qed_heff_batch_flops(self.h, C.byref(f), C.byref(b)))
        return f.value, b.value
