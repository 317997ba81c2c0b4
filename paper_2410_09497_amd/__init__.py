"""Matrix-free H(div)-DG Stokes multigrid on MI355X (gfx950).

Python face of libstokesmg: torch provides device memory and streams, the
HIP library does every step.  ``StokesMG`` owns one library handle and its
workspace (a torch uint8 buffer on the device).
"""
import ctypes
import importlib

__all__ = ["StokesMG", "F64", "F32", "StokesMGError", "load_library"]

F64, F32 = 0, 1


def load_library():
    """The ctypes binding; raises ImportError when libstokesmg.so is not
    built (there is no fallback path)."""
    return importlib.import_module(__name__ + "._lib")


_lib = None


class StokesMGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libstokesmg error {code}: {msg}")
        self.code = code


def _torch():
    import torch
    return torch


class StokesMG:
    def __init__(self, n_cells, k, n_levels=None, penalty_factor=2.0, device="cuda:0", cg_rtol=1e-13,
                 cg_max_it=200):
        global _lib
        _lib = load_library()
        torch = _torch()
        if n_levels is None:
            n_levels = n_cells.bit_length()          # down to 1^3
        cfg = _lib.Config(n_cells, k, n_levels, penalty_factor, cg_rtol, cg_max_it)
        h = ctypes.c_void_p()
        rc = _lib.lib.stokesmg_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != 0:
            raise StokesMGError(rc, "stokesmg_create rejected the configuration")
        self._h = h
        self._L = _lib            # keeps the library alive until this handle is released
        self._destroy = _lib.lib.stokesmg_destroy   # still callable during interpreter shutdown
        self.n_cells, self.k, self.n_levels = n_cells, k, n_levels
        self.device = torch.device(device)
        nb = ctypes.c_size_t()
        self._check(_lib.lib.stokesmg_workspace_size(h, ctypes.byref(nb)))
        self.workspace = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            self._check(_lib.lib.stokesmg_set_workspace(h, self.workspace.data_ptr(), self.workspace.numel(),
                                                       self._stream()))

    def __del__(self):
        h = getattr(self, "_h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and h.value and destroy is not None:
            destroy(h)
            self._h = None

    def _stream(self):
        return _torch().cuda.current_stream(self.device).cuda_stream

    def _check(self, rc):
        if rc != 0:
            msg = _lib.lib.stokesmg_last_error(self._h).decode()
            raise StokesMGError(rc, msg)

    @staticmethod
    def _dtype_code(t):
        torch = _torch()
        if t.dtype == torch.float64:
            return F64
        if t.dtype == torch.float32:
            return F32
        raise TypeError("vectors must be float64 or float32")

    def sizes(self, level=-1):
        level = level % self.n_levels
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(_lib.lib.stokesmg_sizes(self._h, level, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def ndof(self, level=-1):
        return self.sizes(level)[2]

    def _vec(self, t, level, name):
        if not t.is_contiguous() or t.device != self.device or t.numel() != self.ndof(level):
            raise ValueError(f"{name}: need a contiguous {self.ndof(level)}-vector on {self.device}")

    def apply(self, x, y=None, level=-1):
        """y = K x on ``level`` (default finest)."""
        level = level % self.n_levels
        if y is None:
            y = _torch().empty_like(x)
        self._vec(x, level, "x")
        self._vec(y, level, "y")
        self._check(_lib.lib.stokes_apply(self._h, level, self._dtype_code(x), x.data_ptr(), y.data_ptr(),
                                          self._stream()))
        return y

    def residual(self, b, x, r=None, level=-1):
        """r = b - K x on ``level``."""
        level = level % self.n_levels
        if r is None:
            r = _torch().empty_like(x)
        for t, nm in ((b, "b"), (x, "x"), (r, "r")):
            self._vec(t, level, nm)
        if not (b.dtype == x.dtype == r.dtype):
            raise TypeError("b, x, r must share a dtype")
        self._check(_lib.lib.stokes_residual(self._h, level, self._dtype_code(x), b.data_ptr(), x.data_ptr(),
                                             r.data_ptr(), self._stream()))
        return r

    def smooth(self, x, b, level=-1, sweeps=1):
        """x <- S(x, b): ``sweeps`` colourized vertex-patch sweeps, in place."""
        level = level % self.n_levels
        self._vec(x, level, "x")
        self._vec(b, level, "b")
        if x.dtype != b.dtype:
            raise TypeError("x and b must share a dtype")
        self._check(_lib.lib.patch_smooth(self._h, level, self._dtype_code(x), x.data_ptr(), b.data_ptr(), sweeps,
                                          self._stream()))
        return x

    def smooth_noalloc(self, x, b, level=-1, sweeps=1):
        """patch_smooth_noalloc: the same sweeps with the library's static
        device scratch instead of the workspace; returns the local CG
        iterations of the call (synchronizes the stream)."""
        level = level % self.n_levels
        self._vec(x, level, "x")
        self._vec(b, level, "b")
        if x.dtype != b.dtype:
            raise TypeError("x and b must share a dtype")
        it = ctypes.c_int64(-1)
        self._check(_lib.lib.patch_smooth_noalloc(self._h, level, self._dtype_code(x), x.data_ptr(), b.data_ptr(),
                                                  sweeps, ctypes.byref(it), self._stream()))
        return it.value

    def cg_stats(self, reset=True):
        """(local CG iterations, local solves) since the last reset."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        self._check(_lib.lib.stokesmg_cg_stats(self._h, ctypes.byref(a), ctypes.byref(b), int(reset),
                                               self._stream()))
        return a.value, b.value

    def vcycle(self, b, x=None):
        """x = P^{-1} b: one V-cycle on the finest level (dtype of b)."""
        if x is None:
            x = _torch().empty_like(b)
        self._vec(b, -1, "b")
        self._vec(x, -1, "x")
        self._check(_lib.lib.vcycle(self._h, self._dtype_code(b), b.data_ptr(), x.data_ptr(), self._stream()))
        return x

    def rhs_manufactured(self, level=-1, problem=0):
        """Right-hand side of a manufactured problem (0: the sine/curl solution), FP64."""
        torch = _torch()
        level = level % self.n_levels
        b = torch.empty(self.ndof(level), dtype=torch.float64, device=self.device)
        self._check(_lib.lib.stokesmg_rhs_manufactured(self._h, level, problem, b.data_ptr(), self._stream()))
        return b

    def rhs_fourier(self, seed, level=-1, n_modes=8):
        """Right-hand side of the random smooth force of synth.fourier_modes(seed)."""
        import numpy as np
        from .synth import fourier_modes
        torch = _torch()
        level = level % self.n_levels
        kappa, amp, theta = fourier_modes(seed, n_modes=n_modes)
        kappa = np.ascontiguousarray(kappa, dtype=np.int32)
        amp = np.ascontiguousarray(amp, dtype=np.float64)
        theta = np.ascontiguousarray(theta, dtype=np.float64)
        b = torch.empty(self.ndof(level), dtype=torch.float64, device=self.device)
        self._check(_lib.lib.stokesmg_rhs_fourier(self._h, level, n_modes, kappa.ctypes.data, amp.ctypes.data,
                                                  theta.ctypes.data, b.data_ptr(), self._stream()))
        return b

    def solve(self, b, rtol=1e-8, max_it=100, restart=30, vcycle_dtype="f64", x=None, allow_notconv=False):
        """FGMRES(restart) preconditioned by the V-cycle; returns (x, info dict)."""
        torch = _torch()
        if b.dtype != torch.float64:
            raise TypeError("b must be float64")
        self._vec(b, -1, "b")
        if x is None:
            x = torch.empty_like(b)
        nb = ctypes.c_size_t()
        vd = F64 if vcycle_dtype == "f64" else F32
        # the basis never needs more vectors than steps
        m = min(restart, max_it)
        self._check(_lib.lib.stokesmg_solve_workspace_size(self._h, m, vd, ctypes.byref(nb)))
        ws = getattr(self, "_solve_ws", None)
        if ws is None or ws.numel() < nb.value:
            self._solve_ws = None
            ws = self._solve_ws = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        info = _lib.Info()
        rc = _lib.lib.solve(self._h, b.data_ptr(), x.data_ptr(), rtol, max_it, restart, vd, ws.data_ptr(),
                            ws.numel(), ctypes.byref(info), self._stream())
        if rc != 0 and not (allow_notconv and rc == _lib.ENOTCONV):
            self._check(rc)
        hist = [info.history[i] for i in range(min(info.iterations + 1, _lib.MAX_HISTORY))]
        return x, dict(iterations=info.iterations, converged=bool(info.converged), rel_residual=info.rel_residual,
                       nu=info.nu, history=hist, cg_iterations=info.cg_iterations, local_solves=info.local_solves,
                       seconds=info.seconds, fallback_iteration=info.fallback_iteration)

    # ------------------------------------------------------------ learned local solver
    def mlp_dims(self):
        """(d, P): patch vector length and parameter count for this degree."""
        d, p = ctypes.c_int64(), ctypes.c_int64()
        self._check(_lib.lib.mlp_dims(self._h, ctypes.byref(d), ctypes.byref(p)))
        return d.value, p.value

    def mlp_setup(self, max_rows):
        """Allocates the MLP workspace (torch buffer) for batches of max_rows rows."""
        torch = _torch()
        nb = ctypes.c_size_t()
        self._check(_lib.lib.mlp_workspace_size(self._h, int(max_rows), ctypes.byref(nb)))
        self.mlp_workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        self._check(_lib.lib.mlp_set_workspace(self._h, self.mlp_workspace.data_ptr(), self.mlp_workspace.numel(),
                                               int(max_rows)))
        self.mlp_rows = int(max_rows)

    def mlp_init(self, seed=0):
        self._check(_lib.lib.mlp_init(self._h, int(seed), self._stream()))

    def mlp_get_state(self):
        """(state, step): state = params | Adam m | Adam v (float32 device tensor)."""
        torch = _torch()
        _, P = self.mlp_dims()
        st = torch.empty(3 * P, dtype=torch.float32, device=self.device)
        step = ctypes.c_int64()
        self._check(_lib.lib.mlp_get_state(self._h, st.data_ptr(), ctypes.byref(step), self._stream()))
        return st, step.value

    def mlp_set_state(self, state, step=0):
        torch = _torch()
        _, P = self.mlp_dims()
        if state.dtype != torch.float32 or state.numel() != 3 * P or state.device != self.device:
            raise ValueError(f"state must be a float32 tensor of {3 * P} entries on {self.device}")
        state = state.contiguous()
        self._check(_lib.lib.mlp_set_state(self._h, state.data_ptr(), int(step), self._stream()))

    @staticmethod
    def _mode(mode):
        return {"bf16": 0, "f32": 1}[mode]

    def _rows(self, t, name):
        torch = _torch()
        d, _ = self.mlp_dims()
        if t.dtype != torch.float32 or t.dim() != 2 or t.shape[1] != d or not t.is_contiguous() \
                or t.device != self.device:
            raise ValueError(f"{name} must be a contiguous float32 [rows x {d}] tensor on {self.device}")

    def mlp_forward(self, X, mode="bf16"):
        torch = _torch()
        self._rows(X, "X")
        Y = torch.empty_like(X)
        self._check(_lib.lib.mlp_forward(self._h, self._mode(mode), X.data_ptr(), Y.data_ptr(), X.shape[0],
                                         self._stream()))
        return Y

    def mlp_backward(self, X, T, mode="bf16"):
        """(grads, loss): gradient of mean((net(X) - T)^2) and the loss (device tensors)."""
        torch = _torch()
        self._rows(X, "X")
        self._rows(T, "T")
        _, P = self.mlp_dims()
        g = torch.empty(P, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        self._check(_lib.lib.mlp_backward(self._h, self._mode(mode), X.data_ptr(), T.data_ptr(), X.shape[0],
                                          g.data_ptr(), loss.data_ptr(), self._stream()))
        return g, loss

    def mlp_adam_step(self, grads, lr):
        self._check(_lib.lib.mlp_adam_step(self._h, grads.data_ptr(), float(lr), self._stream()))

    def mlp_collect_pairs(self, b, X, T, n=0, x=None):
        """One FP64 V-cycle for b capturing interior-patch pairs into rows n.. of X, T;
        returns (new n, x)."""
        torch = _torch()
        self._vec(b, -1, "b")
        self._rows(X, "X")
        self._rows(T, "T")
        if x is None:
            x = torch.empty_like(b)
        nn = ctypes.c_int64(int(n))
        self._check(_lib.lib.mlp_collect_pairs(self._h, b.data_ptr(), x.data_ptr(), X.data_ptr(), T.data_ptr(),
                                               min(X.shape[0], T.shape[0]), ctypes.byref(nn), self._stream()))
        return nn.value, x

    def mlp_train(self, X, T, n=None, epochs=1, batch=4096, lr=1e-3, seed=0, mode="bf16"):
        """Trains on rows 0..n-1; returns the per-epoch mean losses."""
        self._rows(X, "X")
        self._rows(T, "T")
        n = X.shape[0] if n is None else int(n)
        hist = (ctypes.c_float * max(epochs, 1))()
        self._check(_lib.lib.mlp_train(self._h, self._mode(mode), X.data_ptr(), T.data_ptr(), n, int(epochs),
                                       int(batch), float(lr), int(seed), hist, self._stream()))
        return [hist[i] for i in range(epochs)]

    def set_local_solver(self, solver="exact", mode="bf16", damping=1.0):
        """exact (Schur CG), mlp, mlp_warm, direct, or exact_bf16 (Schur CG with
        the in-plane eigenbasis products on the matrix cores; FP32 cycles)."""
        codes = {"exact": 0, "mlp": 1, "mlp_warm": 2, "direct": 3, "exact_bf16": 4}
        self._check(_lib.lib.stokesmg_set_local_solver(self._h, codes[solver], self._mode(mode), float(damping)))

    def l2_error(self, x, level=-1):
        """(||u - u_h||, ||p - p_h||) of the FP64 level vector x against the
        manufactured sine problem (Gauss k+3 per direction, zero-mean pressures)."""
        level = level % self.n_levels
        self._vec(x, level, "x")
        eu, ep = ctypes.c_double(), ctypes.c_double()
        self._check(_lib.lib.stokesmg_l2_error(self._h, level, 0, x.data_ptr(), ctypes.byref(eu), ctypes.byref(ep),
                                               self._stream()))
        return eu.value, ep.value

    def direct_matrix(self, patch_type=0):
        """The Direct solver's normalized map of one patch type (host, FP64,
        [out][in]); type t_x + 3 t_y + 9 t_z with t_d = 0 inside, 1 at the
        lower and 2 at the upper boundary, 27 for the single patch of n = 2."""
        import numpy as np
        d, _ = self.mlp_dims()
        M = np.empty((d, d), dtype=np.float64)
        self._check(_lib.lib.stokesmg_direct_matrix(self._h, int(patch_type), M.ctypes.data))
        return M

    def direct_setup(self):
        """Uploads the Direct solver's matrix into the MLP workspace (mlp_setup first)."""
        self._check(_lib.lib.stokesmg_direct_setup(self._h, self._stream()))

    def set_fallback(self, rho_ref):
        self._check(_lib.lib.stokesmg_set_fallback(self._h, float(rho_ref)))

    def set_smoothing(self, pre=1, post=1):
        """Smoothing sweeps of the V-cycle before and after the coarse correction."""
        self._check(_lib.lib.stokesmg_set_smoothing(self._h, int(pre), int(post)))
