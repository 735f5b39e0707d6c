"""Python binding of libftafqmc: ph-FT-AFQMC slice propagation for the uniform electron gas on MI355X.

Argument marshalling only: every step of the path runs in the HIP kernels of
libftafqmc.so (built by paper_2012_12228_amd/build.py).  torch supplies device
memory (the workspace and all inputs/outputs) and the stream.  The functions
carry the names of the C ABI declared in include/ftafqmc.h; `Context` bundles
them for one handle.  There is no fallback: without the built library every
call raises.
"""
import ctypes
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libftafqmc.so")

FTAFQMC_FP64, FTAFQMC_MIXED = 0, 1
FTAFQMC_C128, FTAFQMC_C64 = 0, 1
WALKER_ALIVE, WALKER_KILLED, WALKER_NUMERIC = 0, 1, 2
FTAFQMC_CHECKPOINT = 1     # params flag: record the path for ftafqmc_backward
FTAFQMC_OVERLAP = 2        # params flag: two walker groups on two streams
FTAFQMC_GRAPH = 4          # params flag: replay whole-path propagation from a captured HIP graph
FTAFQMC_TRIAL_THF = 8      # params flag: thermal Hartree-Fock trial instead of the free-electron one
FTAFQMC_MODIFIED_OVERLAP = 16     # params flag: constraint from the modified overlap ratio (eq. ztfix)
FTAFQMC_MEASURE_EVERY_SLICE = 32  # params flag: an energy record after every slice
FTAFQMC_LOW_RANK = 64      # params flag: low-rank truncation of the Green's function solve (eq. thresh)
LOW_RANK_THRESHOLD = 1e-6  # FTAFQMC_LOW_RANK_THRESHOLD
FTAFQMC_BF16_SPLIT = 128   # params flag (mixed only): propagator products on BF16 matrix cores, split operands
FTAFQMC_PROFILE_ONLY = 256  # ftafqmc_profile: record only the classes in the low bits
FROZEN_PATH = 0            # ftafqmc_backward modes: shifted fields held fixed
PATHWISE = 1               #   raw fields held fixed, the force bias follows G_k
POP_COMB, POP_PAIR_BRANCH = 0, 1   # ftafqmc_population_control methods
MU_BRACKET_FIT, MU_NEWTON = 0, 1   # ftafqmc_tune_mu methods
STATUS = {0: "OK", -1: "E_ARG", -2: "E_HIP", -3: "E_NUMERIC", -4: "E_STATE", -5: "E_UNSUPPORTED"}

ABI_SYMBOLS = ["ftafqmc_workspace_bytes", "ftafqmc_init_ueg", "ftafqmc_init_ueg_static", "ftafqmc_query",
               "ftafqmc_reset", "ftafqmc_propagate", "ftafqmc_greens", "ftafqmc_energy", "ftafqmc_records",
               "ftafqmc_backward", "ftafqmc_kink_flags", "ftafqmc_lowrank_ranks", "ftafqmc_population_control", "ftafqmc_record_stats",
               "ftafqmc_density_correlation", "ftafqmc_qvectors", "ftafqmc_set_mu", "ftafqmc_tune_mu",
               "ftafqmc_system_times", "ftafqmc_profile",
               "ftafqmc_last_error", "ftafqmc_destroy"]
STATIC_WORKSPACE_BYTES = 64 << 20   # FTAFQMC_STATIC_WORKSPACE_BYTES
PROF_CLASSES = ["gemm", "elim", "greens_transpose", "weight_forcebias", "coef_gather", "stabilise", "energy",
                "backward"]


class Params(ctypes.Structure):
    _fields_ = [("n_elec", ctypes.c_int), ("rs", ctypes.c_double), ("theta", ctypes.c_double),
                ("nmax2", ctypes.c_int), ("dtau", ctypes.c_double), ("stab_every", ctypes.c_int),
                ("n_walkers", ctypes.c_int), ("mu", ctypes.c_double), ("kscale", ctypes.c_double),
                ("precision", ctypes.c_int), ("flags", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("n_q", ctypes.c_int), ("n_slices", ctypes.c_int),
                ("n_walkers", ctypes.c_int), ("slice", ctypes.c_int), ("n_measure", ctypes.c_int),
                ("ld", ctypes.c_int), ("beta", ctypes.c_double), ("dtau", ctypes.c_double),
                ("L", ctypes.c_double), ("omega", ctypes.c_double), ("mu_T", ctypes.c_double),
                ("mu", ctypes.c_double), ("e_madelung", ctypes.c_double),
                ("gemm_tile_chain", ctypes.c_int), ("gemm_tile_apply", ctypes.c_int),
                ("gemm_tile_shapes", ctypes.c_int), ("walker_groups", ctypes.c_int),
                ("gemm_tile_epilogue", ctypes.c_int), ("gemm_tile_horner", ctypes.c_int),
                ("taylor_degree", ctypes.c_int), ("refactor_every", ctypes.c_int)]


class MuResult(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("mu_tilde", ctypes.c_double), ("n_mean", ctypes.c_double),
                ("n_stderr", ctypes.c_double), ("runs", ctypes.c_int)]


_lib_handle = None


def load_library():
    """Load libftafqmc.so (torch must be imported first so that one HIP runtime serves both)."""
    global _lib_handle
    if _lib_handle is not None:
        return _lib_handle
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libftafqmc.so is not built: run `python paper_2012_12228_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    lib.ftafqmc_workspace_bytes.argtypes = [ctypes.POINTER(Params), ip, ctypes.POINTER(sz)]
    lib.ftafqmc_init_ueg.argtypes = [ctypes.POINTER(Params), ip, vp, sz, vp, ctypes.POINTER(vp)]
    lib.ftafqmc_init_ueg_static.argtypes = [ctypes.POINTER(Params), ip, vp, ctypes.POINTER(vp)]
    lib.ftafqmc_query.argtypes = [vp, ip, ctypes.POINTER(Info)]
    lib.ftafqmc_reset.argtypes = [vp, vp]
    lib.ftafqmc_propagate.argtypes = [vp, ctypes.POINTER(vp), ip, vp]
    lib.ftafqmc_greens.argtypes = [vp, ip, vp, ip, vp]
    lib.ftafqmc_energy.argtypes = [vp, ip, vp, vp, vp, vp, vp]
    lib.ftafqmc_records.argtypes = [vp, ip, vp, vp, ctypes.POINTER(ctypes.c_int), vp]
    lib.ftafqmc_backward.argtypes = [vp, ip, ip, vp, vp, vp, vp, vp]
    lib.ftafqmc_kink_flags.argtypes = [vp, ip, ctypes.c_double, vp, vp]
    lib.ftafqmc_lowrank_ranks.argtypes = [vp, ip, vp, ctypes.POINTER(ctypes.c_int), vp]
    lib.ftafqmc_population_control.argtypes = [vp, ip, ip, vp, vp, vp]
    lib.ftafqmc_record_stats.argtypes = [vp, ip, vp, vp, vp]
    lib.ftafqmc_density_correlation.argtypes = [vp, ip, vp, vp, vp]
    lib.ftafqmc_qvectors.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int)]
    lib.ftafqmc_set_mu.argtypes = [vp, ip, ctypes.c_double, vp]
    lib.ftafqmc_system_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.ftafqmc_tune_mu.argtypes = [vp, ip, vp, ip, ctypes.c_double, ctypes.c_double, ip,
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(MuResult), vp]
    lib.ftafqmc_profile.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)]
    lib.ftafqmc_last_error.argtypes = [vp]
    lib.ftafqmc_last_error.restype = ctypes.c_char_p
    lib.ftafqmc_destroy.argtypes = [vp]
    lib.ftafqmc_destroy.restype = None
    for name in ABI_SYMBOLS[:-2]:
        getattr(lib, name).restype = ctypes.c_int
    _lib_handle = lib
    return lib


def _params(sysdef):
    mu = sysdef.get("mu")
    return Params(int(sysdef["n_elec"]), float(sysdef["rs"]), float(sysdef["theta"]), int(sysdef["nmax2"]),
                  float(sysdef["dtau"]), int(sysdef.get("stab_every", 10)), int(sysdef["walkers"]),
                  float("nan") if mu is None else float(mu), float(sysdef.get("kscale", 1.0)),
                  int(sysdef.get("precision", FTAFQMC_FP64)), int(sysdef.get("flags", 0)))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class FtafqmcError(RuntimeError):
    """A C ABI call returned a non-zero ftafqmc_status (in .code)."""

    def __init__(self, code, msg):
        super().__init__("ftafqmc call failed: %s %s" % (STATUS.get(code, code), msg))
        self.code = code


def _check(rc, handle=None):
    if rc != 0:
        # handle None: the message of the last failed initialisation on this thread
        raise FtafqmcError(rc, load_library().ftafqmc_last_error(handle).decode())


# ------------------------------------------------------------ C ABI names ---
def ftafqmc_workspace_bytes(systems):
    arr = (Params * len(systems))(*[_params(s) for s in systems])
    n = ctypes.c_size_t(0)
    _check(load_library().ftafqmc_workspace_bytes(arr, len(systems), ctypes.byref(n)))
    return n.value


def ftafqmc_init_ueg(systems, workspace, device):
    arr = (Params * len(systems))(*[_params(s) for s in systems])
    h = ctypes.c_void_p(0)
    _check(load_library().ftafqmc_init_ueg(arr, len(systems), _ptr(workspace), workspace.numel(),
                                           _stream(device), ctypes.byref(h)))
    return h


def ftafqmc_init_ueg_static(systems, device):
    """Initialise with the library's static device workspace (no device allocation)."""
    arr = (Params * len(systems))(*[_params(s) for s in systems])
    h = ctypes.c_void_p(0)
    _check(load_library().ftafqmc_init_ueg_static(arr, len(systems), _stream(device), ctypes.byref(h)))
    return h


def ftafqmc_query(handle, sys=0):
    info = Info()
    _check(load_library().ftafqmc_query(handle, sys, ctypes.byref(info)), handle)
    return {f: getattr(info, f) for f, _ in Info._fields_}


def ftafqmc_reset(handle, device):
    _check(load_library().ftafqmc_reset(handle, _stream(device)), handle)


def ftafqmc_propagate(handle, fields, n_slices, device):
    for f in fields:
        if f.dtype != torch.complex128 or not f.is_contiguous() or f.device.type != "cuda":
            raise ValueError("fields must be contiguous complex128 CUDA tensors")
    ptrs = (ctypes.c_void_p * len(fields))(*[f.data_ptr() for f in fields])
    _check(load_library().ftafqmc_propagate(handle, ptrs, int(n_slices), _stream(device)), handle)


def ftafqmc_greens(handle, sys, out, device):
    """out: contiguous complex128 or complex64 CUDA tensor of shape [W][M][M] of system `sys`."""
    codes = {torch.complex128: FTAFQMC_C128, torch.complex64: FTAFQMC_C64}
    if out.dtype not in codes:
        raise ValueError("ftafqmc_greens: out must be complex128 or complex64, not %s" % out.dtype)
    if out.device.type != "cuda" or not out.is_contiguous():
        raise ValueError("ftafqmc_greens: out must be a contiguous CUDA tensor")
    inf = ftafqmc_query(handle, sys)
    if tuple(out.shape) != (inf["n_walkers"], inf["M"], inf["M"]):
        raise ValueError("ftafqmc_greens: out must have shape %s" % ((inf["n_walkers"], inf["M"], inf["M"]),))
    _check(load_library().ftafqmc_greens(handle, sys, _ptr(out), codes[out.dtype], _stream(device)), handle)
    return out


def ftafqmc_energy(handle, sys, local, mean, logw, status, device):
    _check(load_library().ftafqmc_energy(handle, sys, _ptr(local), _ptr(mean), _ptr(logw), _ptr(status),
                                         _stream(device)), handle)


def ftafqmc_records(handle, sys, trace, logw, n_rec, device):
    slices = (ctypes.c_int * max(1, n_rec))()
    _check(load_library().ftafqmc_records(handle, sys, _ptr(trace), _ptr(logw), slices, _stream(device)), handle)
    return [slices[i] for i in range(n_rec)]


def ftafqmc_backward(handle, sys, mode, cot, jac, grad, walker, device):
    _check(load_library().ftafqmc_backward(handle, sys, mode, _ptr(cot), _ptr(jac), _ptr(grad), _ptr(walker),
                                           _stream(device)), handle)


def ftafqmc_kink_flags(handle, sys, threshold, flags, device):
    _check(load_library().ftafqmc_kink_flags(handle, sys, float(threshold), _ptr(flags), _stream(device)), handle)


def ftafqmc_lowrank_ranks(handle, sys, m_right, n_slices, device):
    m_left = (ctypes.c_int * (n_slices + 1))()
    _check(load_library().ftafqmc_lowrank_ranks(handle, sys, _ptr(m_right), m_left, _stream(device)), handle)
    return list(m_left)


def ftafqmc_population_control(handle, sys, method, uniforms, parent, device):
    _check(load_library().ftafqmc_population_control(handle, sys, method, _ptr(uniforms), _ptr(parent),
                                                     _stream(device)), handle)


def ftafqmc_record_stats(handle, sys, stats, average, device):
    _check(load_library().ftafqmc_record_stats(handle, sys, _ptr(stats), _ptr(average), _stream(device)), handle)


def ftafqmc_density_correlation(handle, sys, walker, mean, device):
    _check(load_library().ftafqmc_density_correlation(handle, sys, _ptr(walker), _ptr(mean), _stream(device)), handle)


def ftafqmc_qvectors(handle, sys, n_q):
    buf = (ctypes.c_int * (3 * n_q))()
    _check(load_library().ftafqmc_qvectors(handle, sys, buf), handle)
    return [tuple(buf[3 * q:3 * q + 3]) for q in range(n_q)]


def ftafqmc_system_times(handle, n_sys):
    ms = (ctypes.c_double * n_sys)()
    _check(load_library().ftafqmc_system_times(handle, ms), handle)
    return list(ms)


def ftafqmc_set_mu(handle, sys, mu, device):
    _check(load_library().ftafqmc_set_mu(handle, sys, float(mu), _stream(device)), handle)


def ftafqmc_tune_mu(handle, sys, fields, method, n_target, tol, max_runs, device):
    trace = (ctypes.c_double * (4 * max_runs))()
    res = MuResult()
    _check(load_library().ftafqmc_tune_mu(handle, sys, _ptr(fields), method, float(n_target), float(tol), int(max_runs),
                                          trace, ctypes.byref(res), _stream(device)), handle)
    out = {f: getattr(res, f) for f, _ in MuResult._fields_}
    out["trace"] = [tuple(trace[4 * i:4 * i + 4]) for i in range(res.runs)]
    return out


def ftafqmc_profile(handle, enable, classes=None):
    """enable=True starts event timing (every class, or only the class names in `classes`);
    enable=False stops and returns {class: (ms, launches)}."""
    n = len(PROF_CLASSES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_longlong * n)()
    code = 0
    if enable:
        code = 1
        if classes is not None:
            code = FTAFQMC_PROFILE_ONLY
            for c in classes:
                code |= 1 << PROF_CLASSES.index(c)
    _check(load_library().ftafqmc_profile(handle, code, ms, cnt), handle)
    if enable:
        return None
    return {PROF_CLASSES[i]: (ms[i], cnt[i]) for i in range(n)}


def ftafqmc_destroy(handle):
    load_library().ftafqmc_destroy(handle)


# ------------------------------------------------------------- convenience ---
class Context:
    """One library handle over one or more UEG systems, with its torch workspace."""

    def __init__(self, systems, device="cuda:0", static_workspace=False):
        """static_workspace: use ftafqmc_init_ueg_static (the library's own device array, no
        allocation) instead of a torch workspace."""
        if isinstance(systems, dict):
            systems = [systems]
        self.systems = [dict(s) for s in systems]
        self.device = torch.device(device)
        self.handle = None
        load_library()
        if static_workspace:
            self.workspace = None
            with torch.cuda.device(self.device):
                self.handle = ftafqmc_init_ueg_static(self.systems, self.device)
        else:
            nbytes = ftafqmc_workspace_bytes(self.systems)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self.workspace.data_ptr()) % 256
            self.workspace = self.workspace[off:off + nbytes]
            self.handle = ftafqmc_init_ueg(self.systems, self.workspace, self.device)
        self.infos = [ftafqmc_query(self.handle, i) for i in range(len(self.systems))]

    def info(self, sys=0):
        return ftafqmc_query(self.handle, sys)

    def reset(self):
        ftafqmc_reset(self.handle, self.device)

    def propagate(self, fields, n_slices=None):
        if isinstance(fields, torch.Tensor):
            fields = [fields]
        for i, f in enumerate(fields):
            inf = self.infos[i]
            want = (inf["n_walkers"], inf["n_slices"], inf["n_q"])
            if tuple(f.shape) != want:
                raise ValueError("fields of system %d must have shape %s" % (i, want))
        if n_slices is None:
            n_slices = max(inf["n_slices"] for inf in self.infos)
        ftafqmc_propagate(self.handle, fields, n_slices, self.device)
        self._fields = fields        # held until the next call: the pathwise backward re-reads them

    def greens(self, sys=0, dtype=torch.complex128):
        inf = self.infos[sys]
        out = torch.empty((inf["n_walkers"], inf["M"], inf["M"]), dtype=dtype, device=self.device)
        return ftafqmc_greens(self.handle, sys, out, self.device)

    def energy(self, sys=0):
        W = self.infos[sys]["n_walkers"]
        local = torch.empty((W, 4), dtype=torch.complex128, device=self.device)
        mean = torch.empty(4, dtype=torch.complex128, device=self.device)
        logw = torch.empty(W, dtype=torch.float64, device=self.device)
        status = torch.empty(W, dtype=torch.int32, device=self.device)
        ftafqmc_energy(self.handle, sys, local, mean, logw, status, self.device)
        return dict(local=local, mean=mean, logw=logw, status=status)

    def records(self, sys=0):
        inf = self.info(sys)
        n, W = inf["n_measure"], inf["n_walkers"]
        trace = torch.empty((max(n, 1), W, 4), dtype=torch.complex128, device=self.device)
        logw = torch.empty((max(n, 1), W), dtype=torch.float64, device=self.device)
        slices = ftafqmc_records(self.handle, sys, trace, logw, n, self.device)
        return dict(slices=slices, trace=trace[:n], logw=logw[:n])

    def backward(self, sys=0, cot=None, mode=FROZEN_PATH):
        """Derivatives at tau = beta in (mu, lambda) (the system needs flags=FTAFQMC_CHECKPOINT):
        FROZEN_PATH holds the shifted fields fixed, PATHWISE the raw fields (the force bias then
        follows G_k; the path must have been propagated from one field buffer).

        Returns dict(jac [4] complex128 = d<E>/dmu, d<N>/dmu, d<E>/dlambda, d<N>/dlambda,
        walker [W][6] complex128 = (d ln w, dE, dN) along mu then lambda, and
        grad [2] float64 = cot . Re(jac) per parameter when cot (dL/dRe<E>, dL/dRe<N>) is given).
        """
        W = self.infos[sys]["n_walkers"]
        jac = torch.empty(4, dtype=torch.complex128, device=self.device)
        walker = torch.empty((W, 6), dtype=torch.complex128, device=self.device)
        grad = None
        if cot is not None:
            cot = torch.as_tensor(cot, dtype=torch.float64, device=self.device).contiguous()
            grad = torch.empty(2, dtype=torch.float64, device=self.device)
        ftafqmc_backward(self.handle, sys, mode, cot, jac, grad, walker, self.device)
        return dict(jac=jac, walker=walker, grad=grad)

    def lowrank_ranks(self, sys=0):
        """(m_L [n+1] list, m_R [W][n+1] int32 tensor) of a FTAFQMC_LOW_RANK system at every
        Green's function formation (index 0: the initial one, k: after slice k)."""
        inf = self.infos[sys]
        m_right = torch.empty((inf["n_walkers"], inf["n_slices"] + 1), dtype=torch.int32, device=self.device)
        m_left = ftafqmc_lowrank_ranks(self.handle, sys, m_right, inf["n_slices"], self.device)
        return m_left, m_right

    def kink_flags(self, threshold, sys=0):
        """int32 [W]: 1 where the walker's recorded path had cos(theta_k) < threshold on a slice
        it survived (its weight is next to the kink of the phaseless kill)."""
        flags = torch.empty(self.infos[sys]["n_walkers"], dtype=torch.int32, device=self.device)
        ftafqmc_kink_flags(self.handle, sys, threshold, flags, self.device)
        return flags

    def population_control(self, method, uniforms, sys=0):
        """Comb (POP_COMB) or pair branching (POP_PAIR_BRANCH) with the given uniforms (a float64
        CUDA tensor of at least n_walkers values in [0, 1)); returns the parent of every slot."""
        W = self.infos[sys]["n_walkers"]
        u = torch.as_tensor(uniforms, dtype=torch.float64, device=self.device).contiguous()
        if u.numel() < W:
            raise ValueError("population control needs %d uniforms" % W)
        parent = torch.empty(W, dtype=torch.int32, device=self.device)
        ftafqmc_population_control(self.handle, sys, method, u, parent, self.device)
        return parent

    def record_stats(self, sys=0):
        """Per-record weighted statistics [n_rec][8] and their time-slice averages [3]."""
        n = self.info(sys)["n_measure"]
        stats = torch.empty((max(n, 1), 8), dtype=torch.float64, device=self.device)
        avg = torch.empty(3, dtype=torch.float64, device=self.device)
        ftafqmc_record_stats(self.handle, sys, stats, avg, self.device)
        return stats[:n], avg

    def density_correlation(self, sys=0):
        """<rho(Q) rho(-Q)> per walker [W][N_Q] and its weighted mean [N_Q] (complex128); the
        static structure factor is this over N."""
        inf = self.infos[sys]
        walker = torch.empty((inf["n_walkers"], inf["n_q"]), dtype=torch.complex128, device=self.device)
        mean = torch.empty(inf["n_q"], dtype=torch.complex128, device=self.device)
        ftafqmc_density_correlation(self.handle, sys, walker, mean, self.device)
        return walker, mean

    def system_times(self):
        """Milliseconds of each system's share of the last eager propagate call."""
        return ftafqmc_system_times(self.handle, len(self.systems))

    def set_mu(self, mu, sys=0):
        ftafqmc_set_mu(self.handle, sys, mu, self.device)
        self.infos[sys] = self.info(sys)

    def tune_mu(self, fields, method=MU_BRACKET_FIT, n_target=None, tol=1e-8, max_runs=60, sys=0):
        """Tune mu so that <N> at tau = beta matches n_target (default: the system's N)."""
        if n_target is None:
            n_target = self.systems[sys]["n_elec"]
        out = ftafqmc_tune_mu(self.handle, sys, fields, method, n_target, tol, max_runs, self.device)
        self.infos[sys] = self.info(sys)
        return out

    def qvectors(self, sys=0):
        return ftafqmc_qvectors(self.handle, sys, self.infos[sys]["n_q"])

    def profile(self, enable, classes=None):
        return ftafqmc_profile(self.handle, enable, classes)

    def close(self):
        if getattr(self, "handle", None):
            ftafqmc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FrozenPathMeans(torch.autograd.Function):
    """(mu, lambda) -> (Re<E>, Re<N>) at tau = beta for one UEG system and fixed fields.

    forward runs the whole path on a fresh handle (FP64, path recorded); backward contracts the
    cotangents with the frozen-path derivatives computed by ftafqmc_backward.  mu and kscale are
    0-d float64 tensors; `system` is the dict accepted by Context (mu/kscale/precision/flags
    are taken from here); fields is the complex128 [W][n][N_Q] device tensor.
    """

    @staticmethod
    def forward(ctx, mu, kscale, system, fields):
        return FrozenPathMeans._run(ctx, mu, kscale, system, fields, FROZEN_PATH)

    @staticmethod
    def _run(ctx, mu, kscale, system, fields, mode):
        ctx.mode = mode
        ctx.fields = fields          # the pathwise backward re-reads the path's fields
        sysdef = dict(system)
        sysdef.update(mu=float(mu.detach()), kscale=float(kscale.detach()), precision=FTAFQMC_FP64,
                      flags=FTAFQMC_CHECKPOINT)
        c = Context(sysdef, device=fields.device)
        c.propagate(fields)
        e = c.energy()
        ctx.context = c
        return e["mean"][2].real.clone(), e["mean"][3].real.clone()

    @staticmethod
    def backward(ctx, gE, gN):
        c = ctx.context
        cot = torch.stack([gE.reshape(()), gN.reshape(())]).to(torch.float64)
        g = c.backward(cot=cot, mode=ctx.mode)["grad"]
        c.close()
        return g[0], g[1], None, None


class PathwiseMeans(FrozenPathMeans):
    """As FrozenPathMeans with the raw fields held fixed (the force bias of every slice follows
    G_k): the derivative that central differences of the whole run in (mu, lambda) measure."""

    @staticmethod
    def forward(ctx, mu, kscale, system, fields):
        return FrozenPathMeans._run(ctx, mu, kscale, system, fields, PATHWISE)


def walker_slices_per_second(systems_info, seconds):
    """Throughput W * n summed over systems."""
    return sum(i["n_walkers"] * i["n_slices"] for i in systems_info) / seconds
