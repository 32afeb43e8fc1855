"""ctypes binding of libbh.so (include/bh.h).

Argument marshalling only: every step of the Barnes-Hut path runs in the HIP
kernels of the library.  PyTorch provides device memory (tensors' data
pointers) and the stream (torch.cuda.current_stream()).  If the library is
not built, loading fails with an error: there is no fallback.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbh.so")

BH_OK, BH_EINVAL, BH_ENOMEM, BH_EHIP, BH_ESTATE, BH_ECAPACITY = 0, -1, -2, -3, -4, -5
FP64, FP32_REL = 0, 1
FLAG_NO_GRAPH, FLAG_BUDGET_MIN, FLAG_PACK_GROUPS = 1, 2, 4
GEOMETRIC, LEARNED = 0, 1
EXPORT = dict(keys=0, perm=1, nodes=2, moments=3, groups=4, lists=5, acc_sorted=6, sorted_pos=7, quad=8,
              node_qn=9, group_extra=10, root_box=11, drift=12)
MLP_NPARAM = 1259
STAGES = ("keys_sort", "tree", "moments", "groups", "walk", "forces", "integrate", "step")

SYMBOLS = ("bh_create", "bh_destroy", "bh_set_params", "bh_build_tree", "bh_make_lists", "bh_forces",
           "bh_step", "bh_step_continue", "bh_direct_sum", "bh_force_timing", "bh_query", "bh_export",
           "bh_export_groups", "bh_stage_times", "bh_autotune", "bh_mlp_collect", "bh_mlp_train",
           "bh_mlp_weights", "bh_mlp_dataset", "bh_mlp_clear", "bh_mlp_set_dataset", "bh_mlp_predict",
           "bh_mlp_gradient", "bh_mlp_adam", "bh_sample_acc", "bh_direct_sum_static", "bh_last_error")


class Params(C.Structure):
    _fields_ = [("theta", C.c_double), ("eps", C.c_double), ("G", C.c_double), ("central_mass", C.c_double),
                ("n_leaf", C.c_int32), ("n_group", C.c_int32), ("precision", C.c_int32),
                ("criterion", C.c_int32), ("theta_min", C.c_double), ("theta_max", C.c_double),
                ("tau", C.c_double), ("flags", C.c_int32), ("r_coll", C.c_double), ("kappa", C.c_double),
                ("eta", C.c_double), ("cyl_radius", C.c_double), ("reuse_drift", C.c_double),
                ("reuse_frac", C.c_double), ("force_tile", C.c_int32)]


class System(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, C.c_void_p) for k in ("x", "y", "z", "vx", "vy", "vz", "m")]


class Accel(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("ax", "ay", "az", "pot")]


class TrainOpts(C.Structure):
    _fields_ = [("iters", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("seed", C.c_uint64), ("init", C.c_int32)]


class Sizes(C.Structure):
    _fields_ = [("n_particles", C.c_int64), ("n_systems", C.c_int32), ("max_level", C.c_int32),
                ("n_nodes", C.c_int64), ("n_groups", C.c_int64), ("n_pc", C.c_int64), ("n_pp", C.c_int64),
                ("interactions", C.c_int64), ("n_group_used", C.c_int32), ("lists_valid", C.c_int32),
                ("interactions_evaluated", C.c_int64), ("force_evaluations", C.c_int64),
                ("tree_builds", C.c_int64), ("drift_rebuilds", C.c_int64), ("host_syncs", C.c_int64),
                ("force_tile", C.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libbh.so.  torch is imported first so that the library binds to
    the HIP runtime torch already loaded (same SONAME)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run python -m paper_1907_02289_amd.build")
    L = C.CDLL(path)
    vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
    L.bh_create.argtypes = [C.POINTER(vp), C.POINTER(Params)]
    L.bh_destroy.argtypes = [vp]
    L.bh_set_params.argtypes = [vp, C.POINTER(Params)]
    L.bh_build_tree.argtypes = [vp, C.POINTER(System), i32, vp]
    L.bh_make_lists.argtypes = [vp, vp]
    L.bh_forces.argtypes = [vp, C.POINTER(Accel), vp]
    L.bh_step.argtypes = [vp, C.POINTER(System), i32, dbl, i32, i32, vp]
    L.bh_step_continue.argtypes = [vp, dbl, i32, i32, vp]
    L.bh_direct_sum.argtypes = [vp, C.POINTER(System), vp, C.c_int64, vp, vp, vp, vp]
    L.bh_direct_sum_static.argtypes = [vp, C.POINTER(System), vp, C.c_int64, vp, vp, vp, vp]
    L.bh_sample_acc.argtypes = [vp, i32, vp, C.c_int64, vp, vp, vp, vp]
    L.bh_force_timing.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), i32]
    L.bh_autotune.argtypes = [vp, C.POINTER(C.c_int32), i32, i32, C.POINTER(C.c_int32), vp]
    L.bh_mlp_collect.argtypes = [vp, i32, i32, vp]
    L.bh_mlp_train.argtypes = [vp, C.POINTER(TrainOpts), C.POINTER(C.c_double), vp]
    L.bh_mlp_weights.argtypes = [vp, vp, vp]
    L.bh_mlp_dataset.argtypes = [vp, C.POINTER(C.c_int64), vp, vp, vp]
    L.bh_mlp_clear.argtypes = [vp]
    L.bh_mlp_set_dataset.argtypes = [vp, C.c_int64, vp, vp, vp]
    L.bh_mlp_predict.argtypes = [vp, vp, C.c_int64, vp, vp]
    L.bh_mlp_gradient.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    L.bh_mlp_adam.argtypes = [vp, vp, C.c_float, C.c_float, C.c_float, C.c_float, vp]
    L.bh_query.argtypes = [vp, C.POINTER(Sizes)]
    L.bh_export.argtypes = [vp, i32, vp, vp]
    L.bh_export_groups.argtypes = [vp, vp, vp, vp]
    L.bh_stage_times.argtypes = [vp, C.POINTER(C.c_double)]
    L.bh_last_error.argtypes = [vp]
    L.bh_last_error.restype = C.c_char_p
    for name in SYMBOLS:
        if name != "bh_last_error":
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


class BHError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"bh status {status}: {msg}")
        self.status = status


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, n=None, what="array"):
    """Device pointer of a contiguous CUDA FP64 tensor (of n elements when n is
    given); anything else raises before the library could read past it."""
    import torch
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{what}: need a contiguous CUDA float64 tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{what}: {t.numel()} elements, expected {n}")
    return C.c_void_p(t.data_ptr())


class Context:
    """One library context (tree, lists and scratch on the current device)."""

    def __init__(self, theta=0.5, eps=1e-3, G=1.0, central_mass=0.0, n_leaf=8, n_group=64,
                 precision=FP64, criterion=GEOMETRIC, theta_min=0.2, theta_max=1.0, tau=1e-3,
                 use_graphs=True, r_coll=0.0, kappa=0.0, eta=0.0, cyl_radius=0.0, reuse_drift=0.0,
                 reuse_frac=0.0, force_tile=0, budget_min=False, pack_groups=False):
        self.L = load_library()
        flags = ((0 if use_graphs else FLAG_NO_GRAPH) | (FLAG_BUDGET_MIN if budget_min else 0)
                 | (FLAG_PACK_GROUPS if pack_groups else 0))
        self.params = Params(theta, eps, G, central_mass, n_leaf, n_group, precision, criterion,
                             theta_min, theta_max, tau, flags, r_coll, kappa, eta,
                             cyl_radius, reuse_drift, reuse_frac, force_tile)
        h = C.c_void_p()
        self._check(self.L.bh_create(C.byref(h), C.byref(self.params)), ctx=None)
        self.h = h
        self._keep = []       # the systems whose arrays bh_step_continue writes

    def _check(self, st, ctx="self"):
        if st != BH_OK:
            msg = self.L.bh_last_error(self.h).decode() if ctx is not None and getattr(self, "h", None) else ""
            raise BHError(st, msg)

    def close(self):
        if getattr(self, "h", None):
            self.L.bh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, **kw):
        old = {k: getattr(self.params, k) for k in kw}
        for k, v in kw.items():
            setattr(self.params, k, v)
        st = self.L.bh_set_params(self.h, C.byref(self.params))
        if st != BH_OK:
            for k, v in old.items():          # the library kept its parameters: so does the mirror
                setattr(self.params, k, v)
        self._check(st)

    @staticmethod
    def _systems(systems):
        arr = (System * len(systems))()
        for k, s in enumerate(systems):
            n = s["x"].numel()
            arr[k].n = n
            for f in ("x", "y", "z", "vx", "vy", "vz", "m"):
                setattr(arr[k], f, _ptr(s.get(f), n, f"system {k} {f}"))
        return arr

    def build_tree(self, systems):
        arr = self._systems(systems)
        self._check(self.L.bh_build_tree(self.h, arr, len(systems), _stream()))
        self._sizes = [s["x"].numel() for s in systems]
        self._keep = list(systems)

    def make_lists(self):
        self._check(self.L.bh_make_lists(self.h, _stream()))

    def forces(self, outs=None):
        """outs: list (one per system) of dicts with ax, ay, az[, pot] tensors, or None."""
        if outs is None:
            self._check(self.L.bh_forces(self.h, None, _stream()))
            return
        sizes = getattr(self, "_sizes", None)
        if sizes is not None and len(outs) != len(sizes):
            raise ValueError(f"{len(outs)} output sets for {len(sizes)} systems")
        arr = (Accel * len(outs))()
        for k, o in enumerate(outs):
            for f in ("ax", "ay", "az", "pot"):
                setattr(arr[k], f, _ptr(o.get(f), sizes[k] if sizes else None, f"output {k} {f}"))
        self._check(self.L.bh_forces(self.h, arr, _stream()))

    def step(self, systems, dt, n_steps, rebuild_every=1):
        arr = self._systems(systems)
        self._check(self.L.bh_step(self.h, arr, len(systems), float(dt), int(n_steps), int(rebuild_every),
                                   _stream()))
        self._sizes = [s["x"].numel() for s in systems]
        self._keep = list(systems)

    def step_continue(self, dt, n_steps, rebuild_every=1):
        self._check(self.L.bh_step_continue(self.h, float(dt), int(n_steps), int(rebuild_every), _stream()))

    def direct_sum(self, system, targets, out):
        """FP64 direct sum for the targets (int64 CUDA tensor) of one system;
        out: dict of ax, ay, az tensors of len(targets)."""
        import torch
        if not (targets.is_cuda and targets.dtype == torch.int64 and targets.is_contiguous()):
            raise TypeError("targets: need a contiguous CUDA int64 tensor")
        arr = self._systems([system])
        nt = targets.numel()
        self._check(self.L.bh_direct_sum(self.h, arr, C.c_void_p(targets.data_ptr()), nt,
                                         _ptr(out["ax"], nt, "ax"), _ptr(out["ay"], nt, "ay"),
                                         _ptr(out["az"], nt, "az"), _stream()))

    def direct_sum_static(self, system, targets, out):
        """bh_direct_sum_static: direct_sum without any device allocation
        (at most 4096 targets)."""
        import torch
        if not (targets.is_cuda and targets.dtype == torch.int64 and targets.is_contiguous()):
            raise TypeError("targets: need a contiguous CUDA int64 tensor")
        arr = self._systems([system])
        nt = targets.numel()
        self._check(self.L.bh_direct_sum_static(self.h, arr, C.c_void_p(targets.data_ptr()), nt,
                                                _ptr(out["ax"], nt, "ax"), _ptr(out["ay"], nt, "ay"),
                                                _ptr(out["az"], nt, "az"), _stream()))

    def sample_acc(self, targets, out, system=0):
        """Accelerations of the last force evaluation at caller indices
        targets (int64 CUDA tensor) of one system into out (dict of ax, ay,
        az tensors of len(targets))."""
        import torch
        if not (targets.is_cuda and targets.dtype == torch.int64 and targets.is_contiguous()):
            raise TypeError("targets: need a contiguous CUDA int64 tensor")
        nt = targets.numel()
        self._check(self.L.bh_sample_acc(self.h, int(system), C.c_void_p(targets.data_ptr()), nt,
                                         _ptr(out["ax"], nt, "ax"), _ptr(out["ay"], nt, "ay"),
                                         _ptr(out["az"], nt, "az"), _stream()))

    def autotune(self, candidates=(64, 128, 256, 512), rebuild_every=4):
        """Group size (returned) and force tile (then in query()["force_tile"])
        by measured time; the context's parameters take both."""
        arr = (C.c_int32 * len(candidates))(*candidates)
        out = C.c_int32()
        self._check(self.L.bh_autotune(self.h, arr, len(candidates), int(rebuild_every), C.byref(out), _stream()))
        self.params.n_group = out.value
        self.params.force_tile = self.query()["force_tile"]
        return out.value

    # ---- learned opening rule
    def mlp_collect(self, max_groups=256, count_cap=65536):
        self._check(self.L.bh_mlp_collect(self.h, int(max_groups), int(count_cap), _stream()))

    def mlp_train(self, iters=2000, batch=4096, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0, init=True):
        o = TrainOpts(int(iters), int(batch), lr, beta1, beta2, eps, int(seed), 1 if init else 0)
        mse = C.c_double()
        self._check(self.L.bh_mlp_train(self.h, C.byref(o), C.byref(mse), _stream()))
        return mse.value

    def mlp_weights(self, set=None):
        w = np.zeros(MLP_NPARAM, np.float32)
        src = None
        if set is not None:
            src = np.ascontiguousarray(set, np.float32)
            if src.size != MLP_NPARAM:
                raise ValueError(f"mlp_weights: {src.size} values, expected {MLP_NPARAM}")
        self._check(self.L.bh_mlp_weights(self.h, w.ctypes.data_as(C.c_void_p),
                                          None if src is None else src.ctypes.data_as(C.c_void_p)))
        return w if set is None else src

    def mlp_dataset(self):
        n = C.c_int64()
        self._check(self.L.bh_mlp_dataset(self.h, C.byref(n), None, None, None))
        pairs = np.zeros((n.value, 2), np.uint32)
        X = np.zeros((n.value, 4), np.float32)
        Y = np.zeros(n.value, np.float32)
        if n.value:
            self._check(self.L.bh_mlp_dataset(self.h, C.byref(n), pairs.ctypes.data_as(C.c_void_p),
                                              X.ctypes.data_as(C.c_void_p), Y.ctypes.data_as(C.c_void_p)))
        return pairs, X, Y

    def mlp_clear(self):
        self._check(self.L.bh_mlp_clear(self.h))

    def mlp_set_dataset(self, X, Y, pairs=None):
        """Replace the training set: features X (n x 4), labels Y (n), and
        optionally the (group, node) pairs (n x 2), all host arrays."""
        X = np.ascontiguousarray(X, np.float32).reshape(-1, 4)
        Y = np.ascontiguousarray(Y, np.float32).reshape(-1)
        if Y.size != X.shape[0]:
            raise ValueError(f"mlp_set_dataset: {X.shape[0]} feature rows, {Y.size} labels")
        P = None
        if pairs is not None:
            P = np.ascontiguousarray(pairs, np.uint32).reshape(-1, 2)
            if P.shape[0] != X.shape[0]:
                raise ValueError(f"mlp_set_dataset: {P.shape[0]} pairs for {X.shape[0]} rows")
        self._check(self.L.bh_mlp_set_dataset(self.h, X.shape[0], None if P is None else P.ctypes.data_as(C.c_void_p),
                                               X.ctypes.data_as(C.c_void_p), Y.ctypes.data_as(C.c_void_p)))

    def mlp_predict(self, X):
        import torch
        X = X.contiguous()
        if not (X.is_cuda and X.dtype == torch.float32 and X.dim() == 2 and X.shape[1] == 4):
            raise TypeError("mlp_predict: need a CUDA float32 tensor of shape (n, 4)")
        out = torch.zeros(X.shape[0], dtype=torch.float32, device=X.device)
        self._check(self.L.bh_mlp_predict(self.h, C.c_void_p(X.data_ptr()), X.shape[0],
                                          C.c_void_p(out.data_ptr()), _stream()))
        return out

    def mlp_gradient(self, X, Y):
        import torch
        X, Y = X.contiguous(), Y.contiguous()
        if not (X.is_cuda and Y.is_cuda and X.dtype == torch.float32 and Y.dtype == torch.float32
                and X.dim() == 2 and X.shape[1] == 4 and Y.numel() == X.shape[0]):
            raise TypeError("mlp_gradient: need CUDA float32 X (B x 4) and Y (B)")
        grad = torch.zeros(1249, dtype=torch.float32, device=X.device)
        loss = torch.zeros(1, dtype=torch.float32, device=X.device)
        self._check(self.L.bh_mlp_gradient(self.h, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()),
                                           X.shape[0], C.c_void_p(grad.data_ptr()), C.c_void_p(loss.data_ptr()),
                                           _stream()))
        return grad, loss

    def mlp_adam(self, grad, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam step of the weights with grad (CUDA float32 tensor of 1249)."""
        import torch
        if not (isinstance(grad, torch.Tensor) and grad.is_cuda and grad.dtype == torch.float32
                and grad.is_contiguous() and grad.numel() == 1249):
            raise TypeError("mlp_adam: need a contiguous CUDA float32 tensor of 1249 values")
        self._check(self.L.bh_mlp_adam(self.h, C.c_void_p(grad.data_ptr()), lr, beta1, beta2, eps, _stream()))

    def force_timing(self, reset=True):
        """(total ms, launches) of the force kernel since the last reset."""
        ms, k = C.c_double(), C.c_int64()
        self._check(self.L.bh_force_timing(self.h, C.byref(ms), C.byref(k), 1 if reset else 0))
        return ms.value, k.value

    def query(self):
        s = Sizes()
        self._check(self.L.bh_query(self.h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in Sizes._fields_}

    def export(self, what):
        q = self.query()
        n, nn, ng = q["n_particles"], q["n_nodes"], q["n_groups"]
        if what == "keys":
            out = np.zeros(n, np.uint64)
        elif what == "perm":
            out = np.zeros(n, np.uint32)
        elif what == "nodes":
            out = np.zeros((nn, 8), np.int64)
        elif what == "moments":
            out = np.zeros((nn, 4))
        elif what == "groups":
            out = np.zeros((ng, 4), np.int64)
        elif what in ("acc_sorted", "sorted_pos"):
            out = np.zeros((n, 4))
        elif what == "drift":
            out = np.zeros(nn)
        elif what == "quad":
            out = np.zeros((nn, 6))
        elif what == "node_qn":
            out = np.zeros(nn, np.float32)
        elif what == "group_extra":
            out = np.zeros((ng, 2))
        elif what == "root_box":
            out = np.zeros((q["n_systems"], 4))
        elif what == "lists":
            npc, npp = q["n_pc"], q["n_pp"]
            raw = np.zeros(2 * (ng + 1) * 8 + 4 * (npc + npp) + 8, np.uint8)
            self._check(self.L.bh_export(self.h, EXPORT[what], raw.ctypes.data_as(C.c_void_p), _stream()))
            off = raw[: 2 * (ng + 1) * 8].view(np.int64)
            ids = raw[2 * (ng + 1) * 8: 2 * (ng + 1) * 8 + 4 * (npc + npp)].view(np.uint32)
            return off[: ng + 1].copy(), ids[:npc].copy(), off[ng + 1:].copy(), ids[npc:].copy()
        else:
            raise ValueError(what)
        self._check(self.L.bh_export(self.h, EXPORT[what], out.ctypes.data_as(C.c_void_p), _stream()))
        return out

    def export_groups(self):
        ng = self.query()["n_groups"]
        box = np.zeros((ng, 6), np.int32)
        cen = np.zeros((ng, 3))
        self._check(self.L.bh_export_groups(self.h, box.ctypes.data_as(C.c_void_p),
                                            cen.ctypes.data_as(C.c_void_p), _stream()))
        return box, cen

    def stage_times(self):
        ms = (C.c_double * 8)()
        self._check(self.L.bh_stage_times(self.h, ms))
        return dict(zip(STAGES, list(ms)))


def to_device(system, device="cuda"):
    """numpy System (paper_1907_02289_amd.inputs) -> dict of FP64 device tensors."""
    import torch
    return {k: torch.as_tensor(np.ascontiguousarray(getattr(system, k)), dtype=torch.float64, device=device)
            for k in ("x", "y", "z", "vx", "vy", "vz", "m")}
