"""Python layer over the SORF C ABI.

PyTorch supplies device memory and the current HIP stream; every step of the
computation runs in the HIP library (``libsorf.so``). Tensors passed in must
already live on the GPU with the documented dtype and be contiguous.

Paper: arXiv 2206.01580, Theory section -- RFF feature map and atomic energy
decomposition (``forward``/``predict``), regularised normal equation
(``gram_accumulate``/``solve``), derivative features for forces
(``backward``/``predict`` with Jacobians), SORF operator with per-element
sign diagonals and stacking (``Model``).
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib


def pack_signs(signs_pm1: np.ndarray) -> np.ndarray:
    """+-1 entries [E, T, S, d] -> uint32 words [E, T, S, ceil(d/32)], bit j of
    word j // 32 set when entry j is -1."""
    s = np.asarray(signs_pm1)
    E, T, S, d = s.shape
    W = (d + 31) // 32
    bits = np.zeros((E, T, S, W * 32), dtype=np.uint64)
    bits[..., :d] = (s < 0)
    weights = (np.uint64(1) << np.arange(32, dtype=np.uint64))
    words = (bits.reshape(E, T, S, W, 32) * weights).sum(axis=-1)
    return words.astype(np.uint32)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _need(t: torch.Tensor, dtype, name: str, numel: Optional[int] = None):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")


@dataclass
class Model:
    """Resident SORF parameters: packed sign diagonals and phases on the GPU."""

    d: int
    n_stacks: int
    n_transforms: int
    n_elements: int
    sigma: float
    signs: torch.Tensor   # int32 view of the packed uint32 words
    bias: torch.Tensor    # float32 [E, D]

    @property
    def n_features(self) -> int:
        return self.d * self.n_stacks

    @classmethod
    def from_arrays(cls, signs_pm1: np.ndarray, bias: np.ndarray, sigma: float,
                    device="cuda") -> "Model":
        E, T, S, d = signs_pm1.shape
        packed = pack_signs(signs_pm1)
        return cls(d, S, T, E, float(sigma),
                   torch.from_numpy(packed.view(np.int32)).to(device).contiguous(),
                   torch.from_numpy(np.ascontiguousarray(bias, dtype=np.float32)).to(device))

    @classmethod
    def from_problem(cls, p, device="cuda") -> "Model":
        return cls.from_arrays(p.signs, p.bias, p.sigma, device)

    def c_struct(self) -> _lib.SorfModel:
        return _lib.SorfModel(self.d, self.n_stacks, self.n_transforms, self.n_elements,
                              self.sigma, self.signs.data_ptr(), self.bias.data_ptr())


@dataclass
class Batch:
    """Molecules in CSR form on the GPU."""

    x: torch.Tensor         # float32 [A, d]
    element: torch.Tensor   # int32 [A]
    mol_ptr: torch.Tensor   # int64 [M + 1]

    @property
    def n_atoms(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_mols(self) -> int:
        return int(self.mol_ptr.shape[0] - 1)

    @classmethod
    def from_arrays(cls, x, element, mol_ptr, device="cuda") -> "Batch":
        return cls(torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32)).to(device),
                   torch.as_tensor(np.ascontiguousarray(element, dtype=np.int32)).to(device),
                   torch.as_tensor(np.ascontiguousarray(mol_ptr, dtype=np.int64)).to(device))

    @classmethod
    def from_problem(cls, p, device="cuda") -> "Batch":
        return cls.from_arrays(p.x, p.element, p.mol_ptr, device)

    def c_struct(self, x: Optional[torch.Tensor] = None) -> _lib.SorfBatch:
        xx = self.x if x is None else x
        return _lib.SorfBatch(xx.data_ptr() if xx.numel() else None,
                              self.element.data_ptr() if self.element.numel() else None,
                              self.mol_ptr.data_ptr(), self.n_atoms, self.n_mols)

    def check(self, model: Model):
        _need(self.x, torch.float32, "x", self.n_atoms * model.d)
        _need(self.element, torch.int32, "element", self.n_atoms)
        _need(self.mol_ptr, torch.int64, "mol_ptr")


def forward(model: Model, batch: Batch, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Z [n_mols, D] (sorf_forward)."""
    batch.check(model)
    D = model.n_features
    if out is None:
        out = torch.empty((batch.n_mols, D), dtype=torch.float32, device=batch.x.device)
    _need(out, torch.float32, "Z", batch.n_mols * D)
    lib = _lib.load()
    m, b = model.c_struct(), batch.c_struct()
    _lib.check("sorf_forward", lib.sorf_forward(ctypes.byref(m), ctypes.byref(b),
                                                _ptr(out), _stream()))
    return out


def backward(model: Model, batch: Batch, alpha: torch.Tensor, dE: Optional[torch.Tensor] = None,
             out: Optional[torch.Tensor] = None, x: Optional[torch.Tensor] = None) -> torch.Tensor:
    """dL/dx [n_atoms, d] for L = sum_m dE_m E_m (sorf_backward)."""
    batch.check(model)
    _need(alpha, torch.float32, "alpha", model.n_features)
    if dE is not None:
        _need(dE, torch.float32, "dE", batch.n_mols)
    xx = batch.x if x is None else x
    _need(xx, torch.float32, "x", batch.n_atoms * model.d)
    if out is None:
        out = torch.empty((batch.n_atoms, model.d), dtype=torch.float32, device=xx.device)
    _need(out, torch.float32, "grad_x", batch.n_atoms * model.d)
    lib = _lib.load()
    m, b = model.c_struct(), batch.c_struct(xx)
    _lib.check("sorf_backward", lib.sorf_backward(ctypes.byref(m), ctypes.byref(b), _ptr(alpha),
                                                  _ptr(dE), _ptr(out), _stream()))
    return out


class EnergyGrad:
    """Energies E [n_mols] and dE/dx [n_atoms, d] in one pass over the features
    (sorf_energy_grad), with the workspace kept between calls."""

    def __init__(self, model: Model, device="cuda"):
        self.model = model
        self.device = torch.device(device)
        self.ws = torch.empty(0, dtype=torch.uint8, device=self.device)

    def __call__(self, batch: Batch, alpha: torch.Tensor, E: Optional[torch.Tensor] = None,
                 grad: Optional[torch.Tensor] = None):
        model = self.model
        batch.check(model)
        _need(alpha, torch.float32, "alpha", model.n_features)
        if E is None:
            E = torch.empty(batch.n_mols, dtype=torch.float32, device=self.device)
        if grad is None:
            grad = torch.empty((batch.n_atoms, model.d), dtype=torch.float32, device=self.device)
        _need(E, torch.float32, "E", batch.n_mols)
        _need(grad, torch.float32, "grad_x", batch.n_atoms * model.d)
        lib = _lib.load()
        need = lib.sorf_energy_grad_workspace_bytes(batch.n_atoms)
        if self.ws.numel() < need + 256:
            self.ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        m, b = model.c_struct(), batch.c_struct()
        _lib.check("sorf_energy_grad", lib.sorf_energy_grad(
            ctypes.byref(m), ctypes.byref(b), _ptr(alpha), _ptr(E), _ptr(grad),
            self.ws.data_ptr() + off, need, _stream()))
        return E, grad


def derivative_features(model: Model, batch: Batch, J: torch.Tensor, J_ptr: torch.Tensor,
                        out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """dZ [3 n_atoms, D]: minus the coordinate derivatives of the molecules'
    feature rows, one row per atomic coordinate (sorf_derivative_features)."""
    batch.check(model)
    D = model.n_features
    _need(J, torch.float32, "J")
    _need(J_ptr, torch.int64, "J_ptr", batch.n_mols + 1)
    if out is None:
        out = torch.empty((3 * batch.n_atoms, D), dtype=torch.float32, device=batch.x.device)
    _need(out, torch.float32, "dZ", 3 * batch.n_atoms * D)
    lib = _lib.load()
    m, b = model.c_struct(), batch.c_struct()
    _lib.check("sorf_derivative_features", lib.sorf_derivative_features(
        ctypes.byref(m), ctypes.byref(b), _ptr(J), _ptr(J_ptr), _ptr(out), _stream()))
    return out


class Projector:
    """Per-element projection x_i = rho_i^T U_{e_i} (sorf_project); owns its
    workspace. U: [n_elements, d_rep, d] float32 on the device."""

    def __init__(self, U: torch.Tensor):
        _need(U, torch.float32, "U")
        if U.dim() != 3:
            raise ValueError("U must be [n_elements, d_rep, d]")
        self.U = U
        self.ws = torch.empty(0, dtype=torch.uint8, device=U.device)

    def __call__(self, rho: torch.Tensor, element: torch.Tensor,
                 out: Optional[torch.Tensor] = None) -> torch.Tensor:
        E, d_rep, d = self.U.shape
        A = element.numel()
        _need(rho, torch.float32, "rho", A * d_rep)
        _need(element, torch.int32, "element", A)
        if out is None:
            out = torch.empty((A, d), dtype=torch.float32, device=rho.device)
        _need(out, torch.float32, "x", A * d)
        lib = _lib.load()
        need = lib.sorf_project_workspace_bytes(A, E)
        if self.ws.numel() < need + 256:
            self.ws = torch.empty(need + 256, dtype=torch.uint8, device=rho.device)
        wptr = self.ws.data_ptr() + (-self.ws.data_ptr()) % 256
        _lib.check("sorf_project", lib.sorf_project(
            A, d_rep, _ptr(rho), _ptr(element), E, _ptr(self.U), d, _ptr(out), wptr, need,
            _stream()))
        return out


def projection_fit(sample: torch.Tensor, n_pca: int, out: Optional[torch.Tensor] = None,
                   singular_values: Optional[torch.Tensor] = None):
    """U [d_rep, n_pca] (FP32) and the singular values [n_pca] (FP64) of one
    element's sampled representations [n_samples, d_rep] (sorf_projection_fit)."""
    _need(sample, torch.float32, "sample")
    n, d_rep = sample.shape
    dev = sample.device
    if out is None:
        out = torch.empty((d_rep, n_pca), dtype=torch.float32, device=dev)
    _need(out, torch.float32, "U", d_rep * n_pca)
    if singular_values is None:
        singular_values = torch.empty(n_pca, dtype=torch.float64, device=dev)
    _need(singular_values, torch.float64, "singular_values", n_pca)
    lib = _lib.load()
    need = lib.sorf_projection_fit_workspace_bytes(d_rep)
    ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    wptr = ws.data_ptr() + (-ws.data_ptr()) % 256
    _lib.check("sorf_projection_fit", lib.sorf_projection_fit(
        n, d_rep, _ptr(sample), n_pca, _ptr(out), _ptr(singular_values), wptr, need, _stream()))
    return out, singular_values


def project(rho: torch.Tensor, element: torch.Tensor, U: torch.Tensor,
            out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """x [n_atoms, d] = rho_i^T U_{e_i} (sorf_project)."""
    return Projector(U)(rho, element, out)


def fchl19_params(n2=24, n3=20, eta2=0.32, eta3=2.7, N2=1.8, N3=0.57, c3=13.4, zeta=math.pi,
                  rcut=6.0) -> "_lib.SorfFchl19Params":
    """FCHL19 parameters; the defaults are the paper's energy+force column."""
    return _lib.SorfFchl19Params(int(n2), int(n3), float(eta2), float(eta3), float(N2),
                                 float(N3), float(c3), float(zeta), float(rcut))


def fchl19(R: torch.Tensor, element: torch.Tensor, mol_ptr: torch.Tensor, n_elements: int,
           params=None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """rho [n_atoms, length] FCHL19 representation (sorf_fchl19_forward)."""
    prm = params if params is not None else fchl19_params()
    A = element.numel()
    _need(R, torch.float32, "R", 3 * A)
    _need(element, torch.int32, "element", A)
    _need(mol_ptr, torch.int64, "mol_ptr")
    lib = _lib.load()
    L = lib.sorf_fchl19_length(n_elements, ctypes.byref(prm))
    if L <= 0:
        raise ValueError("invalid FCHL19 parameters or element count")
    if out is None:
        out = torch.empty((A, L), dtype=torch.float32, device=R.device)
    _need(out, torch.float32, "rho", A * L)
    _lib.check("sorf_fchl19_forward", lib.sorf_fchl19_forward(
        _ptr(R), _ptr(element), _ptr(mol_ptr), A, mol_ptr.numel() - 1, n_elements,
        ctypes.byref(prm), _ptr(out), _stream()))
    return out


def fchl19_backward(R: torch.Tensor, element: torch.Tensor, mol_ptr: torch.Tensor,
                    n_elements: int, g: torch.Tensor, params=None,
                    out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """dR [n_atoms, 3] = d(sum_i g_i . rho_i)/dR (sorf_fchl19_backward); forces are -dR."""
    prm = params if params is not None else fchl19_params()
    A = element.numel()
    _need(R, torch.float32, "R", 3 * A)
    _need(element, torch.int32, "element", A)
    _need(mol_ptr, torch.int64, "mol_ptr")
    lib = _lib.load()
    L = lib.sorf_fchl19_length(n_elements, ctypes.byref(prm))
    _need(g, torch.float32, "g", A * L)
    if out is None:
        out = torch.empty((A, 3), dtype=torch.float32, device=R.device)
    _need(out, torch.float32, "dR", 3 * A)
    _lib.check("sorf_fchl19_backward", lib.sorf_fchl19_backward(
        _ptr(R), _ptr(element), _ptr(mol_ptr), A, mol_ptr.numel() - 1, n_elements,
        ctypes.byref(prm), _ptr(g), _ptr(out), _stream()))
    return out


class GramWorkspace:
    """Reusable device workspace for sorf_gram_accumulate (grows on demand)."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = torch.empty(0, dtype=torch.uint8, device=device)

    def get(self, n_rows: int, D: int, precision: str):
        lib = _lib.load()
        if precision == "split":
            need = lib.sorf_gram_split_workspace_bytes(n_rows, D)
        else:
            need = lib.sorf_gram_workspace_bytes(n_rows, D, _lib.GRAM_MODES[precision])
        if need == 0:
            return None, 0
        if self.buf.numel() < need + 256:
            self.buf = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        return self.buf.data_ptr() + (-self.buf.data_ptr()) % 256, need


def gram_accumulate(Z: torch.Tensor, G: torch.Tensor, y: Optional[torch.Tensor] = None,
                    Zty: Optional[torch.Tensor] = None, precision: str = "fp32",
                    scale_exp: int = 0, workspace: Optional[GramWorkspace] = None) -> None:
    """G += Z^T Z on the lower triangle; Zty += Z^T y (sorf_gram_accumulate;
    sorf_gram_accumulate_f64 for precision 'fp64' and sorf_gram_accumulate_split for
    'split', where G and Zty are float64)."""
    M, D = Z.shape
    _need(Z, torch.float32, "Z")
    acc_t = torch.float64 if precision in ("fp64", "split") else torch.float32
    _need(G, acc_t, "G", D * D)
    if y is not None:
        _need(y, torch.float32, "y", M)
        _need(Zty, acc_t, "Zty", D)
    lib = _lib.load()
    if precision == "fp64":
        _lib.check("sorf_gram_accumulate_f64", lib.sorf_gram_accumulate_f64(
            M, D, _ptr(Z), _ptr(y), _ptr(G), _ptr(Zty), _stream()))
        return
    ws = workspace if workspace is not None else GramWorkspace(Z.device)
    wptr, wbytes = ws.get(M, D, precision)
    if precision == "split":
        _lib.check("sorf_gram_accumulate_split", lib.sorf_gram_accumulate_split(
            M, D, _ptr(Z), _ptr(y), _ptr(G), _ptr(Zty), wptr, wbytes, _stream()))
        return
    _lib.check("sorf_gram_accumulate", lib.sorf_gram_accumulate(
        M, D, _ptr(Z), _ptr(y), _lib.GRAM_MODES[precision], scale_exp, _ptr(G), _ptr(Zty),
        wptr, wbytes, _stream()))


def fp16_scale_exp(max_abs: float) -> int:
    """Power-of-two exponent that brings |Z| <= max_abs to at most 2^14, so the
    fp16 hi part stays finite and the lo part keeps its precision."""
    if max_abs <= 0.0:
        return 0
    return int(max(-60, min(60, math.floor(14 - math.log2(max_abs)))))


class Solver:
    """Owns the FP64 workspace of sorf_solve for one system size.

    With ``lookahead=True`` it also owns a ``sorf_solve_streams`` (a second
    stream and two events, created by the library for this object only) and
    runs the two-stream factorisation schedule (``sorf_solve_streamed``);
    otherwise every launch goes to the current stream (``sorf_solve``). The
    results are bitwise the same. One Solver must not be called from two
    threads at once; each thread needs its own."""

    def __init__(self, D: int, device="cuda", lookahead: bool = True):
        lib = _lib.load()
        self.D = D
        nbytes = lib.sorf_solve_workspace_bytes(D)
        if nbytes == 0:
            raise ValueError(f"unsupported system size {D}")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        self.ws_off = (-self.ws.data_ptr()) % 256
        self.nbytes = nbytes
        self.info = torch.zeros(1, dtype=torch.int32, device=device)
        self._streams = None
        if lookahead:
            st = _lib.SorfSolveStreams()
            with torch.cuda.device(self.ws.device):
                _lib.check("sorf_solve_streams_create", lib.sorf_solve_streams_create(
                    ctypes.byref(st)))
            self._streams = st

    def close(self) -> None:
        """Release the side stream and events (also done on garbage collection)."""
        if self._streams is not None:
            st, self._streams = self._streams, None
            _lib.load().sorf_solve_streams_destroy(ctypes.byref(st))

    def __del__(self):
        try:
            self.close()
        except Exception:  # pragma: no cover - interpreter shutdown
            pass

    def __call__(self, G: torch.Tensor, Zty: torch.Tensor, lam: float, n_refine: int = 3,
                 out: Optional[torch.Tensor] = None) -> torch.Tensor:
        D = self.D
        f64 = G.dtype == torch.float64
        _need(G, G.dtype if f64 else torch.float32, "G", D * D)
        _need(Zty, torch.float64 if f64 else torch.float32, "Zty", D)
        if out is None:
            out = torch.empty(D, dtype=torch.float64, device=G.device)
        _need(out, torch.float64, "alpha", D)
        lib = _lib.load()
        args = (D, _ptr(G), _ptr(Zty), float(lam), int(n_refine), _ptr(out), _ptr(self.info),
                self.ws.data_ptr() + self.ws_off, self.nbytes)
        if self._streams is None:
            fn, name = ((lib.sorf_solve_f64, "sorf_solve_f64") if f64
                        else (lib.sorf_solve, "sorf_solve"))
            _lib.check(name, fn(*args, _stream()))
        else:
            fn, name = ((lib.sorf_solve_f64_streamed, "sorf_solve_f64_streamed") if f64
                        else (lib.sorf_solve_streamed, "sorf_solve_streamed"))
            _lib.check(name, fn(*args, ctypes.byref(self._streams), _stream()))
        return out


def solve(G: torch.Tensor, Zty: torch.Tensor, lam: float, n_refine: int = 3):
    """alpha (FP64) and the LAPACK-style info flag (device tensor)."""
    s = Solver(Zty.numel(), device=G.device)
    a = s(G, Zty, lam, n_refine)
    return a, s.info


class Predictor:
    """Energies and forces without forming Z (sorf_predict); owns its workspace."""

    def __init__(self, model: Model, device="cuda"):
        self.model = model
        self.device = device
        self.ws = torch.empty(0, dtype=torch.uint8, device=device)

    def _workspace(self, n_atoms: int, n_mols: int):
        lib = _lib.load()
        m = self.model.c_struct()
        need = lib.sorf_predict_workspace_bytes(ctypes.byref(m), n_atoms, n_mols)
        if self.ws.numel() < need + 256:
            self.ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        return self.ws.data_ptr() + off, need

    def __call__(self, batch: Batch, alpha: torch.Tensor, J: Optional[torch.Tensor] = None,
                 J_ptr: Optional[torch.Tensor] = None, E: Optional[torch.Tensor] = None,
                 F: Optional[torch.Tensor] = None):
        model = self.model
        batch.check(model)
        _need(alpha, torch.float32, "alpha", model.n_features)
        dev = batch.x.device
        if E is None:
            E = torch.empty(batch.n_mols, dtype=torch.float32, device=dev)
        _need(E, torch.float32, "E", batch.n_mols)
        if J is not None:
            _need(J, torch.float32, "J")
            _need(J_ptr, torch.int64, "J_ptr", batch.n_mols + 1)
            if F is None:
                F = torch.empty(3 * batch.n_atoms, dtype=torch.float32, device=dev)
            _need(F, torch.float32, "F", 3 * batch.n_atoms)
        ws, nbytes = self._workspace(batch.n_atoms, batch.n_mols)
        lib = _lib.load()
        m, b = model.c_struct(), batch.c_struct()
        _lib.check("sorf_predict", lib.sorf_predict(
            ctypes.byref(m), ctypes.byref(b), _ptr(alpha), _ptr(J), _ptr(J_ptr), _ptr(E),
            _ptr(F if J is not None else None), ws, nbytes, _stream()))
        return (E, F) if J is not None else E


class ForceContraction:
    """F = -sum_i J_i^T grad_x_i per molecule (sorf_forces); owns its workspace."""

    def __init__(self, device="cuda"):
        self.device = device
        self.ws = torch.empty(0, dtype=torch.uint8, device=device)

    def __call__(self, mol_ptr: torch.Tensor, grad_x: torch.Tensor, J: torch.Tensor,
                 J_ptr: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        _need(mol_ptr, torch.int64, "mol_ptr")
        _need(grad_x, torch.float32, "grad_x")
        if grad_x.dim() != 2:
            raise ValueError("grad_x must be [n_atoms, d]")
        n_atoms, d = int(grad_x.shape[0]), int(grad_x.shape[1])
        n_mols = int(mol_ptr.numel()) - 1
        _need(J, torch.float32, "J")
        _need(J_ptr, torch.int64, "J_ptr", n_mols + 1)
        if out is None:
            out = torch.empty(3 * n_atoms, dtype=torch.float32, device=grad_x.device)
        _need(out, torch.float32, "F", 3 * n_atoms)
        lib = _lib.load()
        need = lib.sorf_forces_workspace_bytes(n_atoms, n_mols)
        if self.ws.numel() < need + 256:
            self.ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        ws = self.ws.data_ptr() + (-self.ws.data_ptr()) % 256
        _lib.check("sorf_forces", lib.sorf_forces(
            d, n_atoms, n_mols, _ptr(mol_ptr), _ptr(grad_x), _ptr(J), _ptr(J_ptr), _ptr(out), ws,
            need, _stream()))
        return out


def forces(mol_ptr: torch.Tensor, grad_x: torch.Tensor, J: torch.Tensor, J_ptr: torch.Tensor,
           out: Optional[torch.Tensor] = None) -> torch.Tensor:
    return ForceContraction(grad_x.device)(mol_ptr, grad_x, J, J_ptr, out)


def predict(model: Model, batch: Batch, alpha: torch.Tensor, J=None, J_ptr=None):
    return Predictor(model, batch.x.device)(batch, alpha, J, J_ptr)


def predict_noalloc(model: Model, batch: Batch, alpha: torch.Tensor, J=None, J_ptr=None,
                    E: Optional[torch.Tensor] = None, F: Optional[torch.Tensor] = None):
    """sorf_predict_noalloc: energies (and forces with J) with the library's fixed
    device scratch as workspace. The outputs E (and F) must be given when the caller
    cannot allocate; calls overlapping on one GPU race on the shared scratch."""
    batch.check(model)
    _need(alpha, torch.float32, "alpha", model.n_features)
    dev = batch.x.device
    if E is None:
        E = torch.empty(batch.n_mols, dtype=torch.float32, device=dev)
    _need(E, torch.float32, "E", batch.n_mols)
    if J is not None:
        _need(J, torch.float32, "J")
        _need(J_ptr, torch.int64, "J_ptr", batch.n_mols + 1)
        if F is None:
            F = torch.empty(3 * batch.n_atoms, dtype=torch.float32, device=dev)
        _need(F, torch.float32, "F", 3 * batch.n_atoms)
    lib = _lib.load()
    m, b = model.c_struct(), batch.c_struct()
    _lib.check("sorf_predict_noalloc", lib.sorf_predict_noalloc(
        ctypes.byref(m), ctypes.byref(b), _ptr(alpha), _ptr(J), _ptr(J_ptr), _ptr(E),
        _ptr(F if J is not None else None), _stream()))
    return (E, F) if J is not None else E


def validate_batch(batch: Batch, n_elements: int) -> int:
    """Device-side CSR / element-range check; returns the flag word (0 = valid)."""
    res = torch.zeros(1, dtype=torch.int32, device=batch.x.device)
    lib = _lib.load()
    b = batch.c_struct()
    _lib.check("sorf_validate_batch", lib.sorf_validate_batch(ctypes.byref(b), n_elements,
                                                              _ptr(res), _stream()))
    return int(res.item())


class SorfEnergy(torch.autograd.Function):
    """E = Z(x) alpha as a differentiable function of x.

    forward: sorf_predict (energies, no Z materialised);
    backward: sorf_backward with the incoming dL/dE as upstream weights."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, model: Model, batch: Batch, alpha: torch.Tensor):
        b = Batch(x.detach().contiguous(), batch.element, batch.mol_ptr)
        E = Predictor(model, x.device)(b, alpha)
        ctx.save_for_backward(x, alpha)
        ctx.model, ctx.batch = model, batch
        return E

    @staticmethod
    def backward(ctx, grad_E: torch.Tensor):
        x, alpha = ctx.saved_tensors
        b = Batch(x.detach().contiguous(), ctx.batch.element, ctx.batch.mol_ptr)
        g = backward(ctx.model, b, alpha, dE=grad_E.contiguous().float())
        return g, None, None, None


def energy(x: torch.Tensor, model: Model, batch: Batch, alpha: torch.Tensor) -> torch.Tensor:
    return SorfEnergy.apply(x, model, batch, alpha)
