"""Host-side tests of the C ABI: the library loads without a GPU, exports every
function ``include/sorf.h`` declares, its structs have the layout the binding
assumes, and invalid arguments are rejected before any HIP call."""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2206_01580_amd import _lib
from paper_2206_01580_amd.sorf import pack_signs, fp16_scale_exp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sorf.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsorf.so is not built (run __graft_entry__.build())")
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sorf_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_binding_table():
    assert declared_functions() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sorf_\w+)", out))
    for name in declared_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None


def test_abi_version(lib):
    assert lib.sorf_abi_version() == 8


def test_struct_layout_matches_c(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "sorf.h"\n'
        "int main(void){\n"
        'printf("%zu %zu %zu %zu %zu\\n", sizeof(sorf_model), offsetof(sorf_model, sigma),'
        " offsetof(sorf_model, signs), offsetof(sorf_model, bias), sizeof(sorf_batch));\n"
        'printf("%zu %zu %zu\\n", offsetof(sorf_batch, mol_ptr), offsetof(sorf_batch, n_atoms),'
        " offsetof(sorf_batch, n_mols));\nreturn 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", f"-I{ROOT}/include", str(src), "-o", str(exe)],
                   check=True)
    a, b = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")[:2]
    M, B = _lib.SorfModel, _lib.SorfBatch
    assert [int(v) for v in a.split()] == [ctypes.sizeof(M), M.sigma.offset, M.signs.offset,
                                           M.bias.offset, ctypes.sizeof(B)]
    assert [int(v) for v in b.split()] == [B.mol_ptr.offset, B.n_atoms.offset, B.n_mols.offset]


def _model(**kw):
    f = dict(d=64, n_stacks=4, n_transforms=3, n_elements=2, sigma=1.0, signs=PTR, bias=PTR)
    f.update(kw)
    return _lib.SorfModel(f["d"], f["n_stacks"], f["n_transforms"], f["n_elements"], f["sigma"],
                          f["signs"], f["bias"])


def _batch(**kw):
    f = dict(x=PTR, element=PTR, mol_ptr=PTR, n_atoms=5, n_mols=2)
    f.update(kw)
    return _lib.SorfBatch(f["x"], f["element"], f["mol_ptr"], f["n_atoms"], f["n_mols"])


# fake, suitably aligned device addresses: every call below fails validation
# before it could touch them
PTR = 4096

BAD_MODELS = [dict(d=3), dict(d=1), dict(d=2048), dict(d=0), dict(n_stacks=0),
              dict(n_transforms=0), dict(n_transforms=4), dict(sigma=0.0), dict(sigma=-1.0),
              dict(sigma=float("nan")), dict(sigma=float("inf")), dict(n_elements=0),
              dict(signs=None), dict(bias=None), dict(d=1024, n_stacks=2048)]


@pytest.mark.parametrize("bad", BAD_MODELS, ids=lambda b: ",".join(f"{k}={v}" for k, v in b.items()))
def test_invalid_models_rejected_before_any_device_call(lib, bad):
    m, b = _model(**bad), _batch()
    assert lib.sorf_forward(ctypes.byref(m), ctypes.byref(b), PTR, None) == _lib.SORF_ERR_INVALID_ARG
    assert lib.sorf_backward(ctypes.byref(m), ctypes.byref(b), PTR, None, PTR, None) == _lib.SORF_ERR_INVALID_ARG
    assert lib.sorf_predict(ctypes.byref(m), ctypes.byref(b), PTR, None, None, PTR, None, PTR, 1 << 30,
                            None) == _lib.SORF_ERR_INVALID_ARG
    assert lib.sorf_predict_workspace_bytes(ctypes.byref(m), 5, 2) == 0


BAD_BATCHES = [dict(n_atoms=-1), dict(n_mols=-1), dict(mol_ptr=None), dict(x=None),
               dict(element=None)]


@pytest.mark.parametrize("bad", BAD_BATCHES, ids=lambda b: ",".join(f"{k}={v}" for k, v in b.items()))
def test_invalid_batches_rejected(lib, bad):
    m, b = _model(), _batch(**bad)
    assert lib.sorf_forward(ctypes.byref(m), ctypes.byref(b), PTR, None) == _lib.SORF_ERR_INVALID_ARG
    assert lib.sorf_validate_batch(ctypes.byref(b), 2, PTR, None) == _lib.SORF_ERR_INVALID_ARG


def test_null_outputs_rejected(lib):
    m, b = _model(), _batch()
    assert lib.sorf_forward(ctypes.byref(m), ctypes.byref(b), None, None) == _lib.SORF_ERR_INVALID_ARG
    assert lib.sorf_backward(ctypes.byref(m), ctypes.byref(b), None, None, PTR, None) == _lib.SORF_ERR_INVALID_ARG
    assert lib.sorf_backward(ctypes.byref(m), ctypes.byref(b), PTR, None, None, None) == _lib.SORF_ERR_INVALID_ARG
    # J without J_ptr, J without F, F without J
    P = lib.sorf_predict
    assert P(ctypes.byref(m), ctypes.byref(b), PTR, PTR, None, PTR, PTR, 256, 1 << 30, None) == _lib.SORF_ERR_INVALID_ARG
    assert P(ctypes.byref(m), ctypes.byref(b), PTR, PTR, PTR, PTR, None, 256, 1 << 30, None) == _lib.SORF_ERR_INVALID_ARG
    assert P(ctypes.byref(m), ctypes.byref(b), PTR, None, None, PTR, PTR, 256, 1 << 30, None) == _lib.SORF_ERR_INVALID_ARG


def test_energy_grad_argument_and_workspace_checks(lib):
    m, b = _model(), _batch()
    EG, Q = lib.sorf_energy_grad, lib.sorf_energy_grad_workspace_bytes
    I, W = _lib.SORF_ERR_INVALID_ARG, _lib.SORF_ERR_WORKSPACE
    assert Q(-1) == 0 and Q(0) == 0 and Q(1) == 256 and Q(65) == 512
    need = Q(b.n_atoms)
    assert EG(ctypes.byref(_model(d=3)), ctypes.byref(b), PTR, PTR, PTR, PTR, need, None) == I
    assert EG(ctypes.byref(m), ctypes.byref(_batch(x=None)), PTR, PTR, PTR, PTR, need, None) == I
    assert EG(ctypes.byref(m), ctypes.byref(b), None, PTR, PTR, PTR, need, None) == I   # alpha
    assert EG(ctypes.byref(m), ctypes.byref(b), PTR, None, PTR, PTR, need, None) == I   # E
    assert EG(ctypes.byref(m), ctypes.byref(b), PTR, PTR, None, PTR, need, None) == I   # grad_x
    assert EG(ctypes.byref(m), ctypes.byref(b), PTR + 4, PTR, PTR, PTR, need, None) == I
    assert EG(ctypes.byref(m), ctypes.byref(b), PTR, PTR, PTR, None, need, None) == W
    assert EG(ctypes.byref(m), ctypes.byref(b), PTR, PTR, PTR, PTR, need - 1, None) == W
    assert EG(ctypes.byref(m), ctypes.byref(b), PTR, PTR, PTR, PTR + 16, need, None) == W


def test_predict_workspace_checks(lib):
    m, b = _model(), _batch()
    need = lib.sorf_predict_workspace_bytes(ctypes.byref(m), 5, 2)
    assert need >= 5 * 4 + 5 * 64 * 4
    P = lib.sorf_predict
    assert P(ctypes.byref(m), ctypes.byref(b), PTR, None, None, PTR, None, None, need, None) == _lib.SORF_ERR_WORKSPACE
    assert P(ctypes.byref(m), ctypes.byref(b), PTR, None, None, PTR, None, 256, need - 1, None) == _lib.SORF_ERR_WORKSPACE
    assert P(ctypes.byref(m), ctypes.byref(b), PTR, None, None, PTR, None, 257, need, None) == _lib.SORF_ERR_WORKSPACE


def test_gram_argument_checks(lib):
    G = lib.sorf_gram_accumulate
    E = _lib.SORF_ERR_INVALID_ARG
    assert G(10, 0, PTR, None, 0, 0, PTR, None, None, 0, None) == E            # D = 0
    assert G(-1, PTR, PTR, None, 0, 0, PTR, None, None, 0, None) == E            # negative rows
    assert G(10, PTR, PTR, None, 6, 0, PTR, None, None, 0, None) == E            # unknown precision
    assert G(10, PTR, PTR, None, 5, 3, PTR, None, None, 0, None) == E            # no scale for fp32 Kahan
    assert G(10, PTR, PTR, None, 0, 3, PTR, None, None, 0, None) == E            # scale only for fp16 modes
    assert G(10, PTR, PTR, None, 2, 61, PTR, None, None, 0, None) == E           # scale range
    assert G(10, PTR, None, None, 0, 0, PTR, None, None, 0, None) == E         # Z missing
    assert G(10, PTR, PTR, None, 0, 0, None, None, None, 0, None) == E         # G missing
    assert G(10, PTR, PTR, PTR, 0, 0, PTR, None, None, 0, None) == E               # y without Zty
    assert G(0, PTR, None, None, 0, 0, PTR, None, None, 0, None) == _lib.SORF_OK  # nothing to do, no launch


def test_gram_workspace_query_and_checks(lib):
    Q = lib.sorf_gram_workspace_bytes
    assert Q(0, 64, 1) == 0 and Q(10, 0, 1) == 0 and Q(-1, 64, 0) == 0 and Q(10, 64, 7) == 0
    fp32, bf, hilo = Q(10, 64, 0), Q(10, 64, 1), Q(10, 64, 3)
    assert 0 < fp32 < bf < hilo
    # 16-bit packing: 64 padded rows (whole 64-row stages) x 256 padded columns x 2 bytes
    # per part
    assert bf - fp32 == 64 * 256 * 2 and hilo - fp32 == 2 * (64 * 256 * 2)
    assert Q(100000, 16384, 3) >= 2 * 100000 * 16384 * 2
    G = lib.sorf_gram_accumulate
    W = _lib.SORF_ERR_WORKSPACE
    assert G(10, 64, PTR, None, 1, 0, PTR, None, None, 0, None) == W            # missing
    assert G(10, 64, PTR, None, 1, 0, PTR, None, PTR, bf - 1, None) == W        # too small
    assert G(10, 64, PTR, None, 1, 0, PTR, None, PTR + 16, bf, None) == W       # not 256-aligned


def test_solve_argument_checks(lib):
    S = lib.sorf_solve
    need = lib.sorf_solve_workspace_bytes(100)
    assert need >= 100 * 100 * 8
    assert lib.sorf_solve_workspace_bytes(0) == 0
    E = _lib.SORF_ERR_INVALID_ARG
    assert S(0, PTR, PTR, 1e-3, 3, PTR, PTR, 256, need, None) == E
    assert S(100, PTR, PTR, -1.0, 3, PTR, PTR, 256, need, None) == E
    assert S(100, PTR, PTR, float("nan"), 3, PTR, PTR, 256, need, None) == E
    assert S(100, PTR, PTR, 1e-3, 17, PTR, PTR, 256, need, None) == E
    assert S(100, None, PTR, 1e-3, 3, PTR, PTR, 256, need, None) == E
    assert S(100, PTR, PTR, 1e-3, 3, PTR, None, 256, need, None) == E
    assert S(100, PTR, PTR, 1e-3, 3, PTR, PTR, 256, need - 1, None) == _lib.SORF_ERR_WORKSPACE
    assert S(100, PTR, PTR, 1e-3, 3, PTR, PTR, None, need, None) == _lib.SORF_ERR_WORKSPACE
    assert S(100, PTR, PTR, 1e-3, 3, PTR, PTR, 264, need, None) == _lib.SORF_ERR_WORKSPACE


def test_gram_split_argument_checks(lib):
    G = lib.sorf_gram_accumulate_split
    need = lib.sorf_gram_split_workspace_bytes(1000, 300)
    # head and tail fragments (1 + 2 + 2 bytes per entry of the padded Z) at least
    assert need >= 1024 * 512 * 5
    assert lib.sorf_gram_split_workspace_bytes(0, 300) == 0
    assert lib.sorf_gram_split_workspace_bytes(10, 0) == 0
    assert lib.sorf_gram_split_workspace_bytes(-1, 300) == 0
    E, W = _lib.SORF_ERR_INVALID_ARG, _lib.SORF_ERR_WORKSPACE
    assert G(-1, 300, PTR, None, PTR, None, PTR, need, None) == E
    assert G(1000, 0, PTR, None, PTR, None, PTR, need, None) == E
    assert G(1000, 300, PTR, None, None, None, PTR, need, None) == E       # no G
    assert G(1000, 300, None, None, PTR, None, PTR, need, None) == E       # no Z
    assert G(1000, 300, PTR, PTR, PTR, None, PTR, need, None) == E         # y without Zty
    assert G(1000, 300, PTR + 4, None, PTR, None, PTR, need, None) == E    # misaligned Z
    assert G(1000, 300, PTR, None, PTR, None, None, need, None) == W
    assert G(1000, 300, PTR, None, PTR, None, PTR, need - 1, None) == W
    assert G(1000, 300, PTR, None, PTR, None, PTR + 16, need, None) == W
    assert G(0, 300, None, None, PTR, None, None, 0, None) == _lib.SORF_OK  # nothing to add


def test_solve_streamed_argument_checks(lib):
    """The streamed solve runs the same host checks as sorf_solve, and rejects a
    resource set with a missing handle, a side stream equal to the call's stream,
    or one event used for both roles -- all before any HIP call."""
    S = lib.sorf_solve_streamed
    need = lib.sorf_solve_workspace_bytes(100)
    E = _lib.SORF_ERR_INVALID_ARG
    ok = _lib.SorfSolveStreams(0x1000, 0x2000, 0x3000)
    args = (100, PTR, PTR, 1e-3, 3, PTR, PTR, 256, need)
    assert S(0, PTR, PTR, 1e-3, 3, PTR, PTR, 256, need, ctypes.byref(ok), None) == E
    assert S(*args[:7], 256, need - 1, ctypes.byref(ok), None) == _lib.SORF_ERR_WORKSPACE
    for bad in (_lib.SorfSolveStreams(None, 0x2000, 0x3000),
                _lib.SorfSolveStreams(0x1000, None, 0x3000),
                _lib.SorfSolveStreams(0x1000, 0x2000, None),
                _lib.SorfSolveStreams(0x1000, 0x2000, 0x2000)):
        assert S(*args, ctypes.byref(bad), None) == E
        assert lib.sorf_solve_f64_streamed(*args, ctypes.byref(bad), None) == E
    # the side stream may not be the call's stream
    assert S(*args, ctypes.byref(ok), 0x1000) == E
    assert lib.sorf_solve_streams_create(None) == E
    assert lib.sorf_solve_streams_destroy(None) == E


def test_solve_streams_struct_layout(tmp_path):
    src = tmp_path / "streams.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "sorf.h"\n'
        "int main(void){\n"
        'printf("%zu %zu %zu %zu\\n", sizeof(sorf_solve_streams), offsetof(sorf_solve_streams, side),'
        " offsetof(sorf_solve_streams, event_fork), offsetof(sorf_solve_streams, event_join));\n"
        "return 0;}\n")
    exe = tmp_path / "streams"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", f"-I{ROOT}/include", str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    S = _lib.SorfSolveStreams
    assert [int(v) for v in out] == [ctypes.sizeof(S), S.side.offset, S.event_fork.offset,
                                     S.event_join.offset]


def test_status_strings(lib):
    for code, name in [(0, "SORF_OK"), (1, "SORF_ERR_INVALID_ARG"), (2, "SORF_ERR_UNSUPPORTED"),
                       (3, "SORF_ERR_DEVICE"), (4, "SORF_ERR_WORKSPACE")]:
        assert lib.sorf_status_string(code).decode() == name


# ------------------------------------------------------------------ host logic
@pytest.mark.parametrize("d", [2, 4, 16, 32, 64, 128, 256])
def test_pack_signs_bit_layout(d):
    rng = np.random.default_rng(d)
    s = (1 - 2 * rng.integers(0, 2, size=(2, 3, 5, d))).astype(np.int8)
    w = pack_signs(s)
    assert w.dtype == np.uint32 and w.shape == (2, 3, 5, (d + 31) // 32)
    for idx in np.ndindex(2, 3, 5):
        for j in range(d):
            bit = (int(w[idx][j // 32]) >> (j % 32)) & 1
            assert bit == (1 if s[idx][j] < 0 else 0)
        if d < 32:
            assert int(w[idx][0]) >> d == 0


def test_fp16_scale_exp():
    assert fp16_scale_exp(0.0) == 0
    for v in (1e-3, 0.3, 1.0, 7.9, 1e3):
        k = fp16_scale_exp(v)
        assert v * 2.0 ** k <= 2 ** 14 < v * 2.0 ** (k + 1)


def test_misaligned_arrays_rejected(lib):
    E = _lib.SORF_ERR_INVALID_ARG
    m, b = _model(bias=PTR + 8), _batch()
    assert lib.sorf_forward(ctypes.byref(m), ctypes.byref(b), PTR, None) == E
    m, b = _model(), _batch(x=PTR + 4)
    assert lib.sorf_forward(ctypes.byref(m), ctypes.byref(b), PTR, None) == E
    m, b = _model(), _batch()
    assert lib.sorf_forward(ctypes.byref(m), ctypes.byref(b), PTR + 4, None) == E
    assert lib.sorf_backward(ctypes.byref(m), ctypes.byref(b), PTR + 4, None, PTR, None) == E
    assert lib.sorf_gram_accumulate(10, 64, PTR + 4, None, 0, 0, PTR, None, None, 0, None) == E


def test_forces_argument_checks(lib):
    F = lib.sorf_forces
    need = lib.sorf_forces_workspace_bytes(5, 2)
    assert need > 0 and lib.sorf_forces_workspace_bytes(-1, 2) == 0
    ok = (64, 5, 2, PTR, PTR, PTR, PTR, PTR, PTR, need, None)
    for i, bad in [(0, 0), (1, -1), (2, -1), (3, None), (2, 0), (4, None), (5, None), (6, None),
                   (7, None)]:
        args = list(ok)
        args[i] = bad
        assert F(*args) == _lib.SORF_ERR_INVALID_ARG, (i, bad)
    args = list(ok)
    args[9] = need - 1
    assert F(*args) == _lib.SORF_ERR_WORKSPACE
    args = list(ok)
    args[8] = PTR + 16
    assert F(*args) == _lib.SORF_ERR_WORKSPACE
    # no atoms: nothing to do, nothing required
    assert F(64, 0, 3, PTR, None, None, None, None, None, 0, None) == _lib.SORF_OK


def test_server_host_checks(lib):
    """sorf_server_*: invalid configurations and pointers are refused before any HIP
    call; queries on a NULL server are refused."""
    m = _model(d=64, n_stacks=4)
    Cfg = _lib.SorfServerConfig
    good = Cfg(1024, 4, 1.0)
    assert lib.sorf_server_workspace_bytes(ctypes.byref(m), ctypes.byref(good)) > 1024 * 64 * 4
    for bad in (Cfg(0, 4, 1.0), Cfg(1024, 0, 1.0), Cfg(1024, 65, 1.0), Cfg(1024, 4, 0.0),
                Cfg(1 << 25, 4, 1.0)):
        assert lib.sorf_server_workspace_bytes(ctypes.byref(m), ctypes.byref(bad)) == 0
    bad_model = _model(d=3)
    assert lib.sorf_server_workspace_bytes(ctypes.byref(bad_model), ctypes.byref(good)) == 0
    h = ctypes.c_void_p(123)
    assert lib.sorf_server_start(ctypes.byref(m), PTR, PTR, PTR, None, ctypes.byref(good), PTR,
                                 1 << 30, None, ctypes.byref(h)) == _lib.SORF_ERR_INVALID_ARG
    assert h.value is None     # cleared on failure
    assert lib.sorf_server_start(ctypes.byref(m), PTR, PTR, PTR, PTR, ctypes.byref(good), None,
                                 1 << 30, None, ctypes.byref(h)) == _lib.SORF_ERR_WORKSPACE
    assert lib.sorf_server_start(ctypes.byref(m), PTR, PTR, PTR, PTR, ctypes.byref(good), 257,
                                 1 << 30, None, ctypes.byref(h)) == _lib.SORF_ERR_WORKSPACE
    t = ctypes.c_int64()
    ao = (ctypes.c_int64 * 2)(0, 5)
    assert lib.sorf_server_submit(None, 1, ao, ao, ctypes.byref(t)) == _lib.SORF_ERR_INVALID_ARG
    assert lib.sorf_server_query(None, 0) == -2
    assert not lib.sorf_server_energies(None, 0)
    assert lib.sorf_server_stop(None, None) == _lib.SORF_ERR_INVALID_ARG
    assert lib.sorf_status_string(_lib.SORF_ERR_BUSY) == b"SORF_ERR_BUSY"
