"""Precision modes of the Gram, end to end through the ridge solve, against
the FP64 oracle on a reduced precision workload (3000 QM9-like molecules,
D = 1024, lambda = 1e-8, 3 refinement steps; kappa(G + lambda I) ~ 8e5).

Each GPU mode's coefficients alpha are scored by the energies Z_ora alpha on
the oracle's own features, relative to the rms of the oracle energies
(err = max |dE| / rms(E)); the bar for the split-precision path is 1e-4.
What the arithmetic fixes is checked:

* split (int8 head + fp16 tail, FP64 G): its error is that of its operand
  representation, which the oracle reproduces exactly (gram_emulated 'split',
  FP64 products and sums: 3.7e-5 on this workload), plus FP32 sums of the tail
  products (2^-7 of G); it must meet the 1e-4 bar and land within 2x of its
  emulation (+1e-5);
* single-product modes (bf16, fp16): likewise within a factor 2 of the
  emulated rounding of their operands;
* modes that store G in FP32 (fp32, fp32_kahan, bf16_hilo, fp16_hilo) cannot
  meet the bar on this workload: rounding the exact FP64 Gram to FP32 and
  solving already gives an energy error above 1e-4 (the oracle computes this
  floor here: 1.3e-4). They are held between half that floor and eight times
  it, and must beat the single fp16 product by 5x;
* FP64: limited by the FP32 features (the GPU computes Z in FP32); bounded
  by 3e-5, ten times the measured 3.2e-6.
On the full precision workload (100,000 molecules, D = 16384) every 16-bit
and split mode must still give a factorable G + lambda I.
"""
import math

import numpy as np
import pytest

from oracle import sorf_oracle as O
from paper_2206_01580_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MODES = ["fp64", "split", "fp32", "fp32_kahan", "bf16_hilo", "fp16_hilo", "fp16", "bf16"]
FP32_G = ["fp32", "fp32_kahan", "bf16_hilo", "fp16_hilo"]


def _scale_exp(D):
    return int(max(-60, min(60, math.floor(14 - math.log2(29 * math.sqrt(2.0 / D))))))


@pytest.fixture(scope="module")
def study():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2206_01580_amd import sorf
    p = W.qm9_like(3000, 8, W.SEED_BASE + 40, "precision-small", sigma=4.0, lam=1e-8)
    D = p.n_features
    Zo = O.molecule_features(p.x, p.element, p.mol_ptr, p.signs, p.bias, p.sigma,
                             chunk_atoms=1 << 20)
    Go, ro = O.gram(Zo, p.y)
    Eo = Zo @ O.solve(Go, ro, p.lam)
    rms = math.sqrt(np.mean(Eo ** 2))
    emulated = {}
    for mode in ("bf16", "fp16", "split"):
        Ge = O.gram_emulated(Zo, mode, _scale_exp(D) if mode == "fp16" else 0)
        emulated[mode] = np.abs(Zo @ O.solve(Ge, ro, p.lam) - Eo).max() / rms
    # FP32 storage floor: the exact FP64 Gram rounded to FP32, then solved
    G32 = Go.astype(np.float32).astype(np.float64)
    emulated["fp32_storage"] = np.abs(Zo @ O.solve(G32, ro, p.lam) - Eo).max() / rms
    model, batch = sorf.Model.from_problem(p), sorf.Batch.from_problem(p)
    Z = sorf.forward(model, batch)
    y = torch.from_numpy(p.y).cuda()
    solver = sorf.Solver(D, device="cuda")
    errs, infos = {}, {}
    for mode in MODES:
        dt = torch.float64 if mode in ("fp64", "split") else torch.float32
        G = torch.zeros(D, D, device="cuda", dtype=dt)
        r = torch.zeros(D, device="cuda", dtype=dt)
        k = _scale_exp(D) if mode.startswith("fp16") else 0
        sorf.gram_accumulate(Z, G, y, r, precision=mode, scale_exp=k)
        a = solver(G, r, p.lam, 3)
        torch.cuda.synchronize()
        infos[mode] = int(solver.info.item())
        errs[mode] = np.abs(Zo @ a.cpu().numpy() - Eo).max() / rms
    print("energy error per mode:", {m: f"{e:.3e}" for m, e in errs.items()},
          "emulated:", {m: f"{e:.3e}" for m, e in emulated.items()})
    return errs, infos, emulated


@pytest.mark.parametrize("mode", MODES)
def test_mode_factors(study, mode):
    assert study[1][mode] == 0


@pytest.mark.parametrize("mode", ["bf16", "fp16"])
def test_single_product_modes_reproduce_their_rounding(study, mode):
    errs, _, emulated = study
    assert 0.5 * emulated[mode] <= errs[mode] <= 2.0 * emulated[mode], (errs[mode], emulated[mode])


def test_split_mode_meets_the_energy_bar(study):
    errs, _, emulated = study
    assert emulated["split"] <= 1e-4
    assert errs["split"] <= 1e-4
    assert errs["split"] <= 2.0 * emulated["split"] + 1e-5


@pytest.mark.parametrize("mode", FP32_G)
def test_fp32_storage_modes(study, mode):
    errs, _, emulated = study
    floor = emulated["fp32_storage"]
    assert floor > 1e-4          # no mode that stores G in FP32 can meet the bar here
    assert 0.5 * floor <= errs[mode] <= 8.0 * floor, (errs[mode], floor)
    assert errs[mode] * 5 <= errs["fp16"]


def test_fp64_mode(study):
    assert study[0]["fp64"] <= 3e-5


def test_precision_workload_factorises_in_every_16bit_mode():
    """The full precision workload (100,000 QM9-like molecules, D = 16384,
    lambda = 1e-8): G + lambda I built by every 16-bit and the split Gram mode still factors.
    Rounding Z to 16 bits keeps the Gram positive semidefinite, so a failure
    here can only come from the FP32 accumulation drifting over a long row
    range (a single matrix-core accumulator over all 100,000 rows did)."""
    from paper_2206_01580_amd import sorf
    p = W.precision_batch(n_mols=100000)
    model, batch = sorf.Model.from_problem(p), sorf.Batch.from_problem(p)
    D = p.n_features
    Z = sorf.forward(model, batch)
    y = torch.from_numpy(p.y).cuda()
    solver = sorf.Solver(D, device="cuda")
    ws = sorf.GramWorkspace("cuda")
    G = torch.empty(D, D, device="cuda")
    r = torch.empty(D, device="cuda")
    infos = {}
    for mode in ("bf16", "fp16", "bf16_hilo", "fp16_hilo"):
        G.zero_()
        r.zero_()
        k = _scale_exp(D) if mode.startswith("fp16") else 0
        sorf.gram_accumulate(Z, G, y, r, precision=mode, scale_exp=k, workspace=ws)
        solver(G, r, p.lam, 1)
        torch.cuda.synchronize()
        infos[mode] = int(solver.info.item())
    del G
    G64 = torch.zeros(D, D, device="cuda", dtype=torch.float64)
    r64 = torch.zeros(D, device="cuda", dtype=torch.float64)
    sorf.gram_accumulate(Z, G64, y, r64, precision="split", workspace=ws)
    solver(G64, r64, p.lam, 1)
    torch.cuda.synchronize()
    infos["split"] = int(solver.info.item())
    assert all(v == 0 for v in infos.values()), infos
