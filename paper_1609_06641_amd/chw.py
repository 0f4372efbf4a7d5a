"""ctypes binding of libchw (argument marshalling only).

Every step of the transform runs in the HIP kernels of libchw.so; this module
only converts Python arguments to the C ABI of include/chw.h.  PyTorch is
used for device memory (tensors) and streams.  If the shared library is not
built, every entry point raises: there is no fallback implementation.
"""

import ctypes
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# CHW_LIBRARY names another build of the library (the host-sanitizer build
# the CPU checks load); by default the in-tree libchw.so
LIB_PATH = os.environ.get("CHW_LIBRARY") or os.path.join(HERE, "libchw.so")

# enums of chw.h
DTYPES = {"f32": 0, "bf16": 1, "f16": 2, "i32": 3, "f64": 4}
NORMS = {"ortho": 0, "none": 1}
STATUS = {0: "CHW_OK", 1: "CHW_ERR_INVALID_ARGUMENT", 2: "CHW_ERR_UNSUPPORTED",
          3: "CHW_ERR_MISALIGNED", 4: "CHW_ERR_OUT_OF_MEMORY", 5: "CHW_ERR_NO_DEVICE",
          6: "CHW_ERR_HIP", 7: "CHW_ERR_DEVICE"}
FLAG_GRAPH = 1 << 0
FLAG_NO_AUTOTUNE = 1 << 1
FLAG_PERSISTENT = 1 << 2
FLAG_MULTI_LAUNCH = 1 << 3
FLAG_ORDER_SEQUENCY = 1 << 4
FLAG_ORDER_NATURAL = 1 << 5
FLAG_THREE_PASS = 1 << 6
ORDERS = {"dyadic": 0, "sequency": FLAG_ORDER_SEQUENCY, "natural": FLAG_ORDER_NATURAL}
SIGN_MODES = {"per_element": 0, "shared": 1}

# symbols declared in include/chw.h: name -> (restype, argtypes)
_VP = ctypes.c_void_p
SIGNATURES = {
    "chw_plan": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int64,
                                ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                ctypes.c_int, ctypes.c_int, ctypes.c_uint32]),
    "chw_workspace_size": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_size_t)]),
    "chw_forward": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "chw_backward": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "chw_forward_noalloc": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "chw_plan_destroy": (ctypes.c_int, [_VP]),
    "chw_plan_set_option": (ctypes.c_int, [_VP, ctypes.c_char_p, ctypes.c_int64]),
    "chw_plan_describe": (ctypes.c_int, [_VP, ctypes.c_char_p, ctypes.c_size_t]),
    "chw_plan_check": (ctypes.c_int, [_VP]),
    "chw_launch_times": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(ctypes.c_int)]),
    "chw_autotune": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.c_int]),
    "chw_forward_signed": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.c_int, ctypes.c_int, _VP]),
    "chw_backward_signed": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.c_int, ctypes.c_int, _VP]),
    "chw_sign_words": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "chw_philox_signs": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, _VP,
                                        _VP]),
    "chw_nodes_forward": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int64, _VP]),
    "chw_nodes_workspace_size": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_size_t)]),
    "chw_haar_forward": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "chw_haar_backward": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "chw_plan_haar_walsh": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int64, ctypes.c_int32,
                                           ctypes.c_int, ctypes.c_int, ctypes.c_uint32]),
    "chw_layout_selfcheck": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t]),
    "chw_tuning_save": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_char_p]),
    "chw_tuning_load": (ctypes.c_int, [ctypes.c_char_p]),
    "chw_tuning_clear": (ctypes.c_int, []),
    "chw_tuning_count": (ctypes.c_int, [ctypes.POINTER(ctypes.c_size_t)]),
    "chw_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "chw_last_error": (ctypes.c_char_p, []),
    "chw_version": (ctypes.c_char_p, []),
}

_lib = None


class CHWError(RuntimeError):
    def __init__(self, status, detail):
        self.status = status
        self.name = STATUS.get(status, "CHW_ERR_%d" % status)
        self.detail = detail
        super().__init__("%s: %s" % (self.name, detail))


def load():
    """Load libchw.so (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libchw.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        # torch ships its own HIP runtime under the same soname; loaded
        # first, it is the one libchw binds to, so the process has a single
        # runtime (loaded after libchw's, torch would map a second one, which
        # then sees no device)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status):
    if status != 0:
        raise CHWError(status, load().chw_last_error().decode())


def version():
    return load().chw_version().decode()


def tuning_save(path, comment=None):
    """Write the process's tuning cache to a text file (chw_tuning_save)."""
    _check(load().chw_tuning_save(os.fsencode(path), None if comment is None else comment.encode()))


def tuning_load(path):
    """Merge a tuning file into the process's cache (chw_tuning_load); plans
    made afterwards without FLAG_NO_AUTOTUNE start from the matching entry."""
    _check(load().chw_tuning_load(os.fsencode(path)))


def tuning_clear():
    _check(load().chw_tuning_clear())


def tuning_count():
    n = ctypes.c_size_t()
    _check(load().chw_tuning_count(ctypes.byref(n)))
    return int(n.value)


def layout_selfcheck():
    """(ok, report) of the host-side check of the kernels' index maps."""
    buf = ctypes.create_string_buffer(1 << 20)
    st = load().chw_layout_selfcheck(buf, len(buf))
    return st == 0, json.loads(buf.value.decode())


def _torch():
    import torch
    return torch


def _stream_ptr(stream, device):
    """hipStream_t of a torch stream, of a raw handle (int), or of the current
    stream of `device` when None."""
    if stream is None:
        stream = _torch().cuda.current_stream(device)
    return stream if isinstance(stream, int) else stream.cuda_stream


_TORCH_DT = {"f32": "float32", "bf16": "bfloat16", "f16": "float16", "i32": "int32",
             "f64": "float64"}


class Plan:
    """A libchw plan for a batch of signals of sizes 2^log2_sizes[i].

    offsets: None (packed back to back) or batch + 1 int64 element offsets.
    dtype: 'f32', 'bf16', 'f16', 'i32' or 'f64'.  norm: 'ortho' or 'none'.
    order: coefficient order 'dyadic' (Paley, eq. 1), 'sequency' (Walsh) or
    'natural' (Sylvester).  three_pass: signals of 2^20 or more take the three
    HBM passes that signals above 2^27 always take (FLAG_THREE_PASS).
    """

    def __init__(self, log2_sizes, dtype="f32", norm="ortho", offsets=None, graph=False,
                 persistent=False, flags=0, order="dyadic", three_pass=False):
        lib = load()
        import numpy as np
        sizes = np.ascontiguousarray(log2_sizes, dtype=np.int32).ravel()
        self.batch = int(sizes.size)
        self.log2_sizes = sizes
        self.dtype = dtype
        self.norm = norm
        offs_arr = None
        if offsets is not None:
            offs_arr = np.ascontiguousarray(offsets, dtype=np.int64).ravel()
            if offs_arr.size != self.batch + 1:
                raise ValueError("offsets needs batch + 1 entries")
        self.offsets = offs_arr
        flags = int(flags) | (FLAG_GRAPH if graph else 0) | (FLAG_PERSISTENT if persistent else 0)
        flags |= FLAG_THREE_PASS if three_pass else 0
        flags |= ORDERS[order]
        self.order = order
        h = _VP()
        _check(lib.chw_plan(ctypes.byref(h), self.batch,
                            sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                            None if offs_arr is None else
                            offs_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            DTYPES[dtype], NORMS[norm], flags))
        self._h = h
        if offs_arr is None:
            self.extent = int(np.sum(np.left_shift(np.int64(1), sizes.astype(np.int64))))
        else:
            self.extent = int(offs_arr[-1])
        self._ws = {}
        # signals in three passes keep two intermediates in the workspace, and
        # the other orders' last passes store outside the blocks they load, so
        # even an out-of-place forward call needs one
        self._ws_always = self.describe()["plan"]["three"] > 0 or order != "dyadic"

    @classmethod
    def haar_walsh(cls, batch, m, dtype="f32", norm="ortho", graph=False):
        """Plan of the Haar-Walsh transform (eq. 4) of `batch` signals of 2^m:
        y = diag(1, H_0, ..., H_{m-1}) w per signal (w: Haar coefficients)."""
        import numpy as np
        lib = load()
        h = _VP()
        _check(lib.chw_plan_haar_walsh(ctypes.byref(h), int(batch), int(m), DTYPES[dtype],
                                       NORMS[norm], FLAG_GRAPH if graph else 0))
        self = cls.__new__(cls)
        per = 1 if m == 0 else m + 1
        sizes = np.tile(np.array([0] + list(range(m)), dtype=np.int32)[:per], int(batch))
        offs = np.concatenate([(np.int64(i) << m) + np.array([0] + [1 << k for k in range(m)],
                                                              dtype=np.int64)[:per]
                               for i in range(int(batch))] + [np.array([int(batch) << m])])
        self.batch, self.log2_sizes, self.dtype, self.norm = int(sizes.size), sizes, dtype, norm
        self.offsets, self.order, self.extent, self._ws, self._h = offs, "dyadic", int(batch) << m, {}, h
        self._ws_always = self.describe()["plan"]["three"] > 0
        return self

    # -- plan queries ---------------------------------------------------------
    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan is closed")
        return self._h

    def workspace_size(self):
        n = ctypes.c_size_t()
        _check(load().chw_workspace_size(self.handle, ctypes.byref(n)))
        return int(n.value)

    def describe(self):
        buf = ctypes.create_string_buffer(1 << 16)
        _check(load().chw_plan_describe(self.handle, buf, len(buf)))
        return json.loads(buf.value.decode())

    def set_option(self, key, value):
        _check(load().chw_plan_set_option(self.handle, key.encode(), int(value)))

    def check(self):
        """Host-side invariants of the plan's work tables (raises on failure)."""
        _check(load().chw_plan_check(self.handle))

    def launch_times(self):
        """Per-launch durations (ms) of the last call; needs option 'timing'."""
        cap = 256
        arr = (ctypes.c_float * cap)()
        n = ctypes.c_int(cap)
        _check(load().chw_launch_times(self.handle, arr, ctypes.byref(n)))
        return [float(arr[i]) for i in range(min(n.value, cap))]

    # -- calls ------------------------------------------------------------------
    def _tensor_check(self, t, name):
        torch = _torch()
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch tensor" % name)
        if t.dtype != getattr(torch, _TORCH_DT[self.dtype]):
            raise TypeError("%s has dtype %s, plan expects %s" % (name, t.dtype, self.dtype))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        if t.device.type != "cuda":
            raise ValueError("%s must live on a GPU device" % name)
        if t.numel() < self.extent:
            raise ValueError("%s holds %d elements, the plan spans %d" % (name, t.numel(), self.extent))

    def _check_workspace(self, workspace, x, need):
        """A caller's workspace must hold `need` bytes, be contiguous and live
        on x's device: the library cannot see a buffer's size, and a short one
        would be written past its end."""
        if workspace is None:
            return None
        torch = _torch()
        if not isinstance(workspace, torch.Tensor):
            raise TypeError("workspace must be a torch tensor")
        if not workspace.is_contiguous():
            raise ValueError("workspace must be contiguous")
        if workspace.device != x.device:
            raise ValueError("workspace is on device %s, the data on %s" % (workspace.device, x.device))
        have = workspace.numel() * workspace.element_size()
        if have < need:
            raise ValueError("workspace holds %d bytes, this plan needs %d (workspace_size())"
                             % (have, need))
        return workspace

    def _workspace(self, device, needed):
        if not needed:
            return None
        nbytes = self.workspace_size()
        key = str(device)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = _torch().empty(max(nbytes, 16), dtype=_torch().uint8, device=device)
            self._ws[key] = ws
        return ws

    def _call(self, fn, x, out, workspace, stream, adjoint, signed=None):
        torch = _torch()
        self._tensor_check(x, "input")
        if out is None:
            out = torch.empty_like(x)
        self._tensor_check(out, "out")
        if workspace is None:
            narrow = self.dtype in ("bf16", "f16")
            rounds = signed[2] if signed else 1
            need = self.workspace_size() > 0 and (adjoint or narrow or rounds > 1 or self._ws_always or
                                                  out.data_ptr() == x.data_ptr())
            workspace = self._workspace(x.device, need)
        else:
            self._check_workspace(workspace, x, self.workspace_size())
        ws_ptr = None if workspace is None else workspace.data_ptr()
        sp = _stream_ptr(stream, x.device)
        if signed is None:
            _check(fn(self.handle, _VP(x.data_ptr()), _VP(out.data_ptr()), _VP(ws_ptr), _VP(sp)))
        else:
            signs, mode, rounds = signed
            _check(fn(self.handle, _VP(x.data_ptr()), _VP(out.data_ptr()), _VP(ws_ptr),
                      _VP(signs.data_ptr()), SIGN_MODES[mode], int(rounds), _VP(sp)))
        return out

    def haar_forward(self, x, out=None, workspace=None, stream=None):
        """out = Psi x per signal (the Haar transform of eq. 2 alone)."""
        torch = _torch()
        if out is None:
            out = torch.empty_like(x)
        if workspace is None:
            workspace = self._workspace(x.device, self.workspace_size() > 0)
        else:
            self._check_workspace(workspace, x, self.workspace_size())
        return self._call(load().chw_haar_forward, x, out, workspace, stream, False)

    def haar_backward(self, g, out=None, workspace=None, stream=None):
        """out = Psi^T g per signal (Haar synthesis)."""
        torch = _torch()
        if out is None:
            out = torch.empty_like(g)
        if workspace is None:
            workspace = self._workspace(g.device, self.workspace_size() > 0)
        else:
            self._check_workspace(workspace, g, self.workspace_size())
        return self._call(load().chw_haar_backward, g, out, workspace, stream, True)

    def sign_words(self, mode="shared"):
        """uint32 words per round of a sign array in layout `mode`."""
        n = ctypes.c_size_t()
        _check(load().chw_sign_words(self.handle, SIGN_MODES[mode], ctypes.byref(n)))
        return int(n.value)

    def philox_signs(self, seed, rounds=1, mode="shared", out=None, device=None, stream=None):
        """int32 tensor of rounds x sign_words(mode) packed sign bits drawn on the
        device from Philox4x64-10 with key (seed, 0) (see chw_philox_signs)."""
        torch = _torch()
        need = int(rounds) * self.sign_words(mode)
        if out is None:
            dev = torch.device("cuda") if device is None else torch.device(device)
            out = torch.empty(max(need, 1), dtype=torch.int32, device=dev)
        self._sign_check(out, mode, rounds)
        sp = _stream_ptr(stream, out.device)
        _check(load().chw_philox_signs(self.handle, SIGN_MODES[mode],
                                       ctypes.c_uint64(int(seed) & (2**64 - 1)), int(rounds),
                                       _VP(out.data_ptr()), _VP(sp)))
        return out

    def nodes_workspace_size(self):
        """Bytes of workspace chw_nodes_forward needs."""
        n = ctypes.c_size_t()
        _check(load().chw_nodes_workspace_size(self.handle, ctypes.byref(n)))
        return int(n.value)

    def nodes_forward(self, x, out=None, workspace=None, chunk=0, stream=None):
        """out = H x per signal evaluated factor by factor (one launch per factor
        of eq. (3), the node decomposition of Sec. 4); for comparison with
        forward(), which computes the same transform."""
        torch = _torch()
        self._tensor_check(x, "input")
        if out is None:
            out = torch.empty_like(x)
        self._tensor_check(out, "out")
        if workspace is None:
            workspace = torch.empty(max(self.nodes_workspace_size(), 16), dtype=torch.uint8,
                                    device=x.device)
        else:
            self._check_workspace(workspace, x, self.nodes_workspace_size())
        sp = _stream_ptr(stream, x.device)
        _check(load().chw_nodes_forward(self.handle, _VP(x.data_ptr()), _VP(out.data_ptr()),
                                        _VP(workspace.data_ptr()), int(chunk), _VP(sp)))
        return out

    def _sign_check(self, signs, mode, rounds):
        torch = _torch()
        if not isinstance(signs, torch.Tensor) or signs.dtype != torch.int32:
            raise TypeError("signs must be an int32 tensor of packed sign bits")
        if not signs.is_contiguous() or signs.device.type != "cuda":
            raise ValueError("signs must be a contiguous GPU tensor")
        need = int(rounds) * self.sign_words(mode)
        if signs.numel() < need:
            raise ValueError("signs holds %d words, %d rounds need %d" % (signs.numel(), rounds, need))

    def forward_signed(self, x, signs, mode="shared", rounds=1, out=None, workspace=None,
                       stream=None):
        """out = H D_k ... H D_1 x per signal; signs: int32 tensor of packed bits
        (rounds x sign_words(mode) words, bit set = sign flip)."""
        self._sign_check(signs, mode, rounds)
        return self._call(load().chw_forward_signed, x, out, workspace, stream, False,
                          (signs, mode, rounds))

    def backward_signed(self, g, signs, mode="shared", rounds=1, out=None, workspace=None,
                        stream=None):
        """out = D_1 H^T ... D_k H^T g per signal (adjoint of forward_signed)."""
        self._sign_check(signs, mode, rounds)
        return self._call(load().chw_backward_signed, g, out, workspace, stream, True,
                          (signs, mode, rounds))

    def forward(self, x, out=None, workspace=None, stream=None):
        """out = H x for every signal (H'x in the unnormalized form)."""
        return self._call(load().chw_forward, x, out, workspace, stream, False)

    def forward_noalloc(self, x, out, stream=None):
        """out = H x through chw_forward_noalloc: the intermediate lives in the
        library's static device scratch, and the call allocates nothing.  `out`
        is required (this method allocates nothing either); the plan's tables
        must already be on the device (one forward/backward call there)."""
        self._tensor_check(x, "input")
        self._tensor_check(out, "out")
        if out.device != x.device:
            raise ValueError("out is on device %s, the input on %s" % (out.device, x.device))
        sp = _stream_ptr(stream, x.device)
        _check(load().chw_forward_noalloc(self.handle, _VP(x.data_ptr()), _VP(out.data_ptr()),
                                          _VP(sp)))
        return out

    def backward(self, g, out=None, workspace=None, stream=None):
        """out = H^T g for every signal: the reversed cascade of transposed factors,
        which in the dyadic order gives the forward's bits, so by default the
        library runs the forward launches (option "adjoint" = 1: the synthesis
        kernels)."""
        return self._call(load().chw_backward, g, out, workspace, stream, True)

    def autotune(self, x, out, workspace=None, iters=3, stream=None):
        torch = _torch()
        self._tensor_check(x, "input")
        self._tensor_check(out, "out")
        if workspace is None:
            workspace = self._workspace(x.device, self.workspace_size() > 0)
        else:
            self._check_workspace(workspace, x, self.workspace_size())
        ws_ptr = None if workspace is None else workspace.data_ptr()
        _check(load().chw_autotune(self.handle, _VP(x.data_ptr()), _VP(out.data_ptr()),
                                   _VP(ws_ptr), _VP(_stream_ptr(stream, x.device)), int(iters)))

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().chw_plan_destroy(self._h)
            self._h = None
        self._ws = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _make_function():
    torch = _torch()

    class CHWFunction(torch.autograd.Function):
        """y = H x per signal; the backward applies H^T through chw_backward."""

        @staticmethod
        def forward(ctx, x, plan):
            ctx.plan = plan
            return plan.forward(x.contiguous())

        @staticmethod
        def backward(ctx, g):
            return ctx.plan.backward(g.contiguous()), None

    return CHWFunction


_fn_cache = None


def chw_function():
    """The torch.autograd.Function wrapping chw_forward / chw_backward."""
    global _fn_cache
    if _fn_cache is None:
        _fn_cache = _make_function()
    return _fn_cache


def transform(x, plan):
    """Differentiable y = H x (applies CHWFunction)."""
    return chw_function().apply(x, plan)


_sfn_cache = None


def signed_function():
    """torch.autograd.Function for y = H D_k ... H D_1 x (fused sign diagonals);
    its backward applies the adjoint through chw_backward_signed."""
    global _sfn_cache
    if _sfn_cache is None:
        torch = _torch()

        class CHWSignedFunction(torch.autograd.Function):
            @staticmethod
            def forward(ctx, x, plan, signs, mode, rounds):
                ctx.plan, ctx.signs, ctx.mode, ctx.rounds = plan, signs, mode, rounds
                return plan.forward_signed(x.contiguous(), signs, mode, rounds)

            @staticmethod
            def backward(ctx, g):
                gx = ctx.plan.backward_signed(g.contiguous(), ctx.signs, ctx.mode, ctx.rounds)
                return gx, None, None, None, None

        _sfn_cache = CHWSignedFunction
    return _sfn_cache


def signed_transform(x, plan, signs, mode="shared", rounds=1):
    """Differentiable y = H D_k ... H D_1 x."""
    return signed_function().apply(x, plan, signs, mode, rounds)
