"""Parity of the HIP path (through the C ABI) against the FP64 CPU oracle."""
import math

import numpy as np
import pytest

from gpu_common import dev, invariant_indices, rel_err, say, torch
from oracle import apply as oapply
from oracle import core as ocore
from oracle_cache import coo, core_zeroed

import paper_2605_28475_amd as wefq
from paper_2605_28475_amd import _lib, synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp64_naive": 1e-12, "fp32": 1e-5, "bf16x3": 3e-5}
_cores = {}


def gpu_core(model, K, L, gamma=None):
    key = (model, K, L, gamma)
    if key not in _cores:
        say(f"[build] {key}")
        _cores[key] = wefq.Core(model, K, L, gamma=gamma, device=0)
    return _cores[key]


def run(core, c, prec):
    d = dev()
    if prec in ("fp64", "fp64_naive"):
        return core.apply_Q(torch.tensor(c, device=d), precision=prec).cpu().numpy()
    out = core.apply_Q(torch.tensor(c, dtype=torch.float32, device=d), precision=prec)
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("K,L,model,gamma", [(3, 3, "hs", 1.0), (3, 3, "mm", 0.0), (3, 3, "vhs", 0.5),
                                             (4, 6, "mm", 0.0), (8, 8, "hs", 1.0), (8, 2, "hs", 1.0)])
def test_core_matches_oracle(K, L, model, gamma):
    say(f"[core] K={K} L={L} {model} gamma={gamma}")
    R = gpu_core(model, K, L, gamma).download_R()
    ref = core_zeroed(K, L, gamma)
    assert rel_err(R, ref) < 1e-12


def test_core_k12_vhs_sampled_channels():
    K = L = 12
    say("[core] K=L=12 vhs 0.5 sampled channels")
    R = gpu_core("vhs", K, L, 0.5).download_R()
    T = coo(L)
    pick = [0, 1, 7, 50, 123, 300, 450, 615]
    ref = ocore.zero_invariants(ocore.core_exact(K, L, 0.5, table=T, subset=pick), T["channels"])
    assert rel_err(R[pick], ref[pick]) < 1e-12


@pytest.mark.parametrize("K,L,model,gamma,B", [(3, 3, "hs", 1.0, 1), (3, 3, "hs", 1.0, 37),
                                               (4, 4, "vhs", 0.5, 21), (8, 8, "hs", 1.0, 19),
                                               (5, 3, "mm", 0.0, 17), (2, 7, "hs", 1.0, 5),
                                               (0, 4, "hs", 1.0, 7), (6, 0, "vhs", 0.5, 9),
                                               (0, 0, "mm", 0.0, 3), (1, 1, "hs", 1.0, 5)])
@pytest.mark.parametrize("prec", ["fp64", "fp64_naive", "fp32", "bf16x3"])
def test_apply_matches_oracle(K, L, model, gamma, B, prec):
    say(f"[apply] K={K} L={L} {model} B={B} {prec}")
    core = gpu_core(model, K, L, gamma)
    c = synth.perturbed_maxwellian(K, L, B, seed=synth.BASE_SEED + 11 * K + L)
    ref = oapply.apply_q(core_zeroed(K, L, gamma), coo(L), c, K)
    q = run(core, c, prec)
    assert rel_err(q, ref) < TOL[prec]
    assert np.all(q[:, invariant_indices(K, L)] == 0.0)


@pytest.mark.parametrize("K", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("slots", [1, 2, 4])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_tile_shapes_match_oracle(K, slots, prec):
    """Every LDS tile layout (odd NK with odd or even H, even NK with or without pad rows)
    at 16-, 8- and 4-cell tiles, against the oracle; the shape is restored afterwards."""
    L = 4
    core = gpu_core("vhs", K, L, 0.5)
    old = core.tune_get(prec)
    say(f"[tiles] K={K} L={L} slots={slots} {prec}")
    core.tune_set(prec, slots, old[1])
    try:
        c = synth.perturbed_maxwellian(K, L, 23, seed=synth.BASE_SEED + 7 * K + slots)
        ref = oapply.apply_q(core_zeroed(K, L, 0.5), coo(L), c, K)
        q = run(core, c, prec)
    finally:
        core.tune_set(prec, *old)
    assert rel_err(q, ref) < TOL[prec]
    assert np.all(q[:, invariant_indices(K, L)] == 0.0)


@pytest.mark.parametrize("K,L", [(4, 4), (12, 12), (16, 16)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_quadratic_homogeneity_bitwise(K, L, prec):
    """Q(2c) = 4 Q(c) exactly: scaling by a power of two commutes with every rounding
    of the path (including the BF16 hi/lo split), so any deviation is a kernel bug."""
    core = gpu_core("vhs", K, L, 0.5)
    c = synth.perturbed_maxwellian(K, L, 9, seed=31 + K)
    say(f"[homogeneity] K={K} L={L} {prec}")
    q1 = run(core, c, prec)
    q2 = run(core, 2.0 * c, prec)
    assert np.array_equal(q2, 4.0 * q1)


@pytest.mark.parametrize("prec", ["fp64", "fp64_naive", "fp32", "bf16x3"])
def test_unit_maxwellian_is_exact_fixed_point(prec):
    K = L = 4
    core = gpu_core("hs", K, L, 1.0)
    q = run(core, synth.unit_maxwellian(K, L, 3), prec)
    assert np.all(q == 0.0)


@pytest.mark.parametrize("prec", ["fp64", "fp64_naive", "fp32", "bf16x3"])
def test_cell_result_independent_of_batch(prec):
    K, L = 6, 6
    core = gpu_core("vhs", K, L, 0.5)
    c = synth.perturbed_maxwellian(K, L, 45, seed=99)
    full = run(core, c, prec)
    for b in (0, 17, 44):
        alone = run(core, c[b:b + 1], prec)
        assert np.array_equal(alone[0], full[b])


@pytest.mark.parametrize("K", [3, 5, 8, 10, 12, 14, 16])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp64"])
def test_wide_workgroups_bitwise_equal(K, prec):
    """The 12- and 16-wave kernel instances (768 and 1,024 threads; the R tile is not hoisted
    from 7x7 quadrants up under 12 waves; 16 waves for quadrants up to 5x5) give bitwise the
    results of the 8-wave instances, at the default tile shape and at one other."""
    core = gpu_core("hs", K, K, 1.0)
    old = core.tune_get(prec)
    B = 40 if K >= 14 else 100
    c = synth.perturbed_maxwellian(K, K, B, seed=synth.BASE_SEED + 900 + K)
    say(f"[wide] K={K} {prec} default {old}")
    try:
        for slots in (old[0], 4 if old[0] != 4 else 2):
            try:
                core.tune_set(prec, slots, 512)
            except wefq.WefqError:
                continue                                  # tile does not fit in LDS
            narrow = run(core, c, prec)
            for block in (768, 1024) if (K + 2) // 2 <= 5 else (768,):
                core.tune_set(prec, slots, block)
                wide = run(core, c, prec)
                assert np.array_equal(narrow, wide), (slots, block)
    finally:
        core.tune_set(prec, *old)


@pytest.mark.parametrize("K,prec", [(12, "fp32"), (12, "fp64"), (16, "fp32"), (16, "bf16x3"), (8, "fp32"),
                                    (8, "bf16x3")])
def test_split_tiles_bitwise_equal(K, prec):
    """A batch large enough for one workgroup per cell tile and small batches whose tiles
    are split over several workgroups give bitwise equal results per cell.  The small FP32
    and BF16x3 batches also take the list of 2-state work units."""
    core = gpu_core("vhs", K, K, 0.5)
    slots, _ = core.tune_get(prec)
    B = 512 * (16 // slots)                       # >= 2 workgroups per CU: no split
    c = synth.perturbed_maxwellian(K, K, B, seed=123 + K)
    say(f"[split] K={K} {prec} B={B} slots={slots}")
    full = run(core, c, prec)
    for lo, hi in ((0, 1), (5, 12), (B - 3, B)):
        part = run(core, c[lo:hi], prec)
        assert np.array_equal(part, full[lo:hi]), (lo, hi)


def test_padded_rows_zero_batch_and_errors():
    K = L = 3
    core = gpu_core("hs", K, L, 1.0)
    d = dev()
    N = core.N
    c = synth.perturbed_maxwellian(K, L, 9, seed=5)
    ref = run(core, c, "fp32")
    fpad = torch.zeros((9, N + 12), dtype=torch.float32, device=d)
    fpad[:, :N] = torch.tensor(c, dtype=torch.float32, device=d)
    qpad = torch.full((9, N + 20), 7.0, dtype=torch.float32, device=d)
    core.apply_Q(fpad[:, :N], out=qpad[:, :N])
    q = qpad.cpu().numpy()
    assert np.array_equal(q[:, :N], ref.astype(np.float32))
    assert np.all(q[:, N:] == 7.0)
    empty = torch.empty((0, N), dtype=torch.float32, device=d)
    assert core.apply_Q(empty).shape == (0, N)
    f = torch.zeros(8 * N + 2, dtype=torch.float32, device=d)
    q = torch.zeros(8 * N + 2, dtype=torch.float32, device=d)
    core.apply_Q(f[1:1 + 4 * N].view(4, N), out=q[1:1 + 4 * N].view(4, N))   # 4-byte aligned is enough
    import ctypes
    from paper_2605_28475_amd import _lib
    st = _lib.lib().wefq_apply_Q(core.handle, _lib.FP32, ctypes.c_void_p(f.data_ptr() + 2),
                                 ctypes.c_void_p(q.data_ptr()), 4, N, N, None)   # 2-byte aligned input
    assert st == _lib.WEFQ_EINVAL
    with pytest.raises(ValueError):
        core.apply_Q(torch.zeros((2, N), dtype=torch.float64, device=d), precision="fp32")


def test_conservation_check_kernel():
    K = L = 5
    core = gpu_core("hs", K, L, 1.0)
    d = dev()
    c = synth.perturbed_maxwellian(K, L, 300, seed=3)
    for prec, dt in (("fp64", torch.float64), ("fp64_naive", torch.float64), ("fp32", torch.float32),
                     ("bf16x3", torch.float32)):
        q = core.apply_Q(torch.tensor(c, dtype=dt, device=d), precision=prec)
        assert core.check_conservation(q, precision=prec) == 0.0
        q[123, 1] = -2.5
        assert core.check_conservation(q, precision=prec) == 2.5


def _wcu(k, l, b0=1 / (4 * math.pi)):
    from scipy.special import eval_legendre, roots_legendre
    t, w = roots_legendre(40)
    c, s = np.sqrt((1 + t) / 2), np.sqrt((1 - t) / 2)
    f = c ** (2 * k + l) * eval_legendre(l, c) + s ** (2 * k + l) * eval_legendre(l, s) - 1 - (k == 0 and l == 0)
    return 2 * math.pi * b0 * float(w @ f)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wcu_spectrum_through_gpu_apply(prec):
    """Linearized Maxwell-molecule operator by polarization: L e_j = [Q(e0+e_j) - Q(e0-e_j)]/2."""
    K = L = 8
    core = gpu_core("mm", K, L, 0.0)
    N = core.N
    e = np.eye(N)
    cells = np.concatenate([e[0] + e, e[0] - e])
    q = run(core, cells, prec)
    Lm = 0.5 * (q[:N] - q[N:]).T            # column j = L e_j
    k, l, _ = synth.mode_kl(K, L)
    lam = np.array([_wcu(a, b) for a, b in zip(k, l)])
    tol = 2e-13 if prec == "fp64" else 5e-6
    assert np.abs(Lm - np.diag(lam)).max() < tol


def test_bkw_identity_through_gpu_apply():
    """Q(c(K))_{k00} = (2 pi b0/3)(1-K) dc_k/dK for the BKW family (Maxwell molecules)."""
    from test_oracle import _bkw_coeffs
    kmax, L = 8, 8
    core = gpu_core("mm", kmax, L, 0.0)
    Ks = np.linspace(0.55, 1.05, kmax + 4)
    coefs = np.array([_bkw_coeffs(Kt, kmax) for Kt in Ks])
    for Kt in (0.6, 0.8, 0.95):
        f = np.zeros((1, core.N))
        f[0, :kmax + 1] = _bkw_coeffs(Kt, kmax)
        q = run(core, f, "fp64")[0]
        dck = np.array([np.polyval(np.polyder(np.polyfit(Ks, coefs[:, k], kmax + 2)), Kt) for k in range(kmax + 1)])
        rhs = (1 - Kt) * dck / 6.0
        assert np.abs(q[:kmax + 1] - rhs).max() < 1e-10
        assert np.abs(q[kmax + 1:]).max() < 1e-13


def test_viscosity_from_gpu_core():
    """Table 4 factors from the GPU-built hard-sphere core."""
    Kmax = 8
    R = gpu_core("hs", Kmax, 2, 1.0).download_R()
    chans = coo(2)["channels"]
    L2 = (R[chans.index((2, 0, 2))][:, 0, :] + R[chans.index((2, 2, 0))][:, :, 0]) / math.sqrt(4 * math.pi)
    fmu = [L2[0, 0] * np.linalg.inv(L2[:K + 1, :K + 1])[0, 0] for K in range(Kmax + 1)]
    for K, val in enumerate([1.000000, 1.014851, 1.015879, 1.016006, 1.016028]):
        assert abs(fmu[K] - val) <= 5e-7
    assert abs(fmu[1] - 205 / 202) < 1e-12


@pytest.mark.parametrize("K,L", [(12, 12), (16, 16), (16, 4), (3, 16)])
def test_large_truncations_fp64_tiled_vs_naive(K, L):
    """Every tile geometry (1, 2 or 4 output states per MFMA column group, two row tiles
    for NK = 17) against the naive FP64 ordering and the FP32 / BF16x3 paths."""
    say(f"[large] K={K} L={L}")
    core = wefq.Core("hs", K, L, device=0)
    c = synth.perturbed_maxwellian(K, L, 23, seed=K * 100 + L)
    ref = run(core, c, "fp64_naive")
    assert rel_err(run(core, c, "fp64"), ref) < 1e-13
    assert rel_err(run(core, c, "fp32"), ref) < 1e-5
    assert rel_err(run(core, c, "bf16x3"), ref) < TOL["bf16x3"]
    core.close()


@pytest.mark.parametrize("K,L,model,gamma", [(12, 12, "vhs", 0.5), (16, 16, "hs", 1.0), (5, 9, "mm", 0.0)])
def test_rotation_equivariance_on_gpu(K, L, model, gamma):
    """Q(D c) = D Q(c) through the GPU path at every precision (no reference values needed)."""
    from rotation import random_rotation, rotate, wigner_blocks
    say(f"[rotation] K={K} L={L} {model}")
    core = gpu_core(model, K, L, gamma)
    blocks = wigner_blocks(L, random_rotation(K + L))
    c = synth.perturbed_maxwellian(K, L, 6, seed=77)
    cr = rotate(c, K, L, blocks)
    for prec, tol in (("fp64", 1e-12), ("fp32", 2 * TOL["fp32"]), ("bf16x3", 2 * TOL["bf16x3"])):
        q = run(core, c, prec)
        qr = run(core, cr, prec)
        assert rel_err(qr, rotate(q, K, L, blocks)) < tol, prec


def test_mode_index_matches_the_layout():
    """wefq_mode_index gives n = (l^2 + l + m) NK + k, the oracle basis order, and refuses modes
    outside the truncation."""
    from oracle import basis
    K, L = 5, 3
    core = wefq.Core("hs", K, L, device=0, precisions=("fp64",))
    for n, (k, l, m) in enumerate(basis.mode_table(K, L)):
        assert core.mode_index(int(k), int(l), int(m)) == n
    for bad in ((K + 1, 0, 0), (0, L + 1, 0), (0, 2, 3), (-1, 0, 0), (0, 1, -2)):
        with pytest.raises(wefq.WefqError) as err:
            core.mode_index(*bad)
        assert err.value.status == _lib.WEFQ_EINVAL
    core.close()


def test_apply_q_argument_errors():
    """Every refusal of wefq_apply_Q through the C-ABI, each checked before any launch (the
    output stays untouched): null handle, unknown or unprepared precision, negative batch,
    null pointers, leading dimensions below N, overlapping input and output."""
    import ctypes
    K = L = 3
    core = wefq.Core("hs", K, L, device=0, precisions=("fp64",))
    N = core.N
    f = torch.tensor(synth.perturbed_maxwellian(K, L, 4, seed=6), device=dev())
    q = torch.full_like(f, 3.0)
    L_ = _lib.lib()
    fp, qp = ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(q.data_ptr())
    h = core.handle
    cases = [
        (None, _lib.FP64, fp, qp, 4, N, N),          # null handle
        (h, 3, fp, qp, 4, N, N),                     # not a precision
        (h, _lib.FP32, fp, qp, 4, N, N),             # precision not prepared
        (h, _lib.FP64, fp, qp, -1, N, N),            # negative batch
        (h, _lib.FP64, None, qp, 4, N, N),           # null input
        (h, _lib.FP64, fp, None, 4, N, N),           # null output
        (h, _lib.FP64, fp, qp, 4, N - 1, N),         # ld_f < N
        (h, _lib.FP64, fp, qp, 4, N, N - 1),         # ld_q < N
        (h, _lib.FP64, fp, fp, 4, N, N),             # Q aliases f
        (h, _lib.FP64, fp, ctypes.c_void_p(f.data_ptr() + 8 * N), 4, N, N),   # overlap
    ]
    for args in cases:
        assert L_.wefq_apply_Q(*args, None) == _lib.WEFQ_EINVAL, args
        assert L_.wefq_last_error()
    torch.cuda.synchronize()
    assert torch.all(q == 3.0)
    assert L_.wefq_apply_Q(h, _lib.FP64, fp, qp, 0, N, N, None) == _lib.WEFQ_OK      # empty batch
    core.close()


def test_binding_refuses_bad_tensors_before_launch():
    """The binding checks every tensor the library would write through a bare pointer: dtype,
    device, unit stride, rows and modes; nothing is launched (the output stays untouched)."""
    K = L = 3
    core = gpu_core("hs", K, L, 1.0)
    d = dev()
    N = core.N
    f32 = torch.tensor(synth.perturbed_maxwellian(K, L, 6, seed=8), dtype=torch.float32, device=d)
    f64 = f32.double()
    good = torch.full((6, N), 5.0, dtype=torch.float32, device=d)
    bad_outs = [torch.empty((6, N), dtype=torch.float64, device=d),          # wrong dtype
                torch.empty((5, N), dtype=torch.float32, device=d),          # too few rows
                torch.empty((6, N + 1), dtype=torch.float32, device=d),      # wrong mode count
                torch.empty((6, 2 * N), dtype=torch.float32, device=d)[:, ::2],   # non-unit stride
                torch.empty((6, N), dtype=torch.float32)]                    # host memory
    for out in bad_outs:
        with pytest.raises(ValueError):
            core.apply_Q(f32, out=out)
    with pytest.raises(ValueError):
        core.apply_Q(f64, out=good, precision="fp64")                         # FP32 out for FP64
    with pytest.raises(ValueError):
        core.apply_Q(f32[:, :N - 1])                                          # f of the wrong size
    with pytest.raises(ValueError):
        core.apply_J(f32, f32, out=bad_outs[1])
    with pytest.raises(ValueError):
        core.check_conservation(torch.zeros((4, N + 3), dtype=torch.float32, device=d))
    with pytest.raises(ValueError):
        wefq.Plan([(core, f32, bad_outs[1])], precision="fp32")
    with pytest.raises(ValueError):
        wefq.Plan([(core, f64, torch.empty_like(f64))], precision="fp32")    # dtype of the plan
    torch.cuda.synchronize()
    assert torch.all(good == 5.0)


@pytest.mark.parametrize("K,model,gamma,pad", [(4, "hs", 1.0, 32), (4, "mm", 0.0, 32), (12, "vhs", 0.5, 16),
                                             (16, "hs", 1.0, 16)])
def test_core_self_convergence_in_padding(K, model, gamma, pad):
    """Section 5.1 (Fig. 2: the core at K = L = 4 converges to FP64 precision as the rules are
    padded).  The rules here are exact for the integrand's degree, so extra points in every
    rule change R only by rounding: sums over 10^4 to 10^5 nodes of terms that cancel, about
    3e-14 of the core's largest entry at K = L = 12; the bound is 1e-13."""
    base_core = gpu_core(model, K, K, gamma)
    base = base_core.download_R()
    padded = wefq.Core(model, K, K, gamma=gamma, device=0, precisions=("fp64",), rad_pad=pad, ang_pad=pad)
    assert padded.info["rad_pad"] == pad and padded.info["quad_nodes"] > base_core.info["quad_nodes"]
    Rp = padded.download_R()
    padded.close()
    err = rel_err(Rp, base)
    per_channel = float(max(np.abs(Rp[c] - base[c]).max() / np.abs(base[c]).max()
                            for c in range(len(base)) if np.abs(base[c]).max() > 0))
    say(f"[padding] K=L={K} {model} pad {pad}: max |R_pad - R_0| / max |R_0| = {err:.2e}, "
        f"worst channel {per_channel:.2e}")
    assert err < 1e-13


def test_binding_works_before_torch_is_imported():
    """A process that uses the binding before importing torch still finds the device: the
    library is loaded after torch's HIP runtime, not beside a second one."""
    import os
    import subprocess
    import sys
    code = ("import paper_2605_28475_amd as w\n"
            "c = w.Core('hs', 2, 2, device=0, precisions=('fp32',))\n"
            "import torch\n"
            "f = torch.zeros((3, c.N), device='cuda'); f[:, 0] = 1.0\n"
            "q = c.apply_Q(f); torch.cuda.synchronize()\n"
            "print('ok', float(q.abs().max()))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    say("[binding] subprocess without torch imported first")
    res = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=240)
    assert res.returncode == 0, res.stderr[-2000:]
    assert res.stdout.strip().startswith("ok")
