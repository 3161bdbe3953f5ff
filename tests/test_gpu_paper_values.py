"""The GPU path against numbers the paper prints, with no oracle in between: the Wang
Chang-Uhlenbeck spectrum of Table 3 and the Chapman-Enskog viscosity factors of Table 4,
both from the linearized operator J(e_000) formed by wefq_apply_J in FP64."""
import math

import numpy as np
import pytest

from gpu_common import dev, say, torch
from oracle_cache import golden

import paper_2605_28475_amd as wefq

pytestmark = pytest.mark.gpu


def linearized(core, cols=None):
    """Columns J(e_000) e_j of the linearized operator (all j, or the given ones), FP64."""
    N = core.N
    cols = np.arange(N) if cols is None else np.asarray(cols)
    c = torch.zeros((len(cols), N), dtype=torch.float64, device=dev())
    c[:, 0] = 1.0
    d = torch.zeros_like(c)
    d[torch.arange(len(cols)), torch.as_tensor(cols, device=dev())] = 1.0
    return core.apply_J(c, d, precision="fp64").cpu().numpy().T        # [N, len(cols)]


def test_table3_wang_chang_uhlenbeck_spectrum():
    """Maxwell molecules, K = 4, L = 6: eigenvalues over |lambda_6|, sorted, against Table 3
    (within the printed difference bounds), and lambda_6 = -4 pi b0 / 3 at b0 = 1/(4 pi)."""
    K, L = 4, 6
    core = wefq.Core("mm", K, L, device=0, precisions=("fp64",))
    Lm = linearized(core)
    ev = np.linalg.eigvals(Lm)
    assert np.abs(ev.imag).max() < 1e-13
    ev = np.sort(ev.real)[::-1]
    ratio = ev / abs(ev[5])
    for first, last, r, bound in golden("table3_wcu.txt"):
        seg = ratio[int(first) - 1:int(last)]
        dev_ = np.abs(seg - float(r)).max()
        say(f"[table3] ratio {r}: max deviation {dev_:.1e} (printed bound {bound})")
        # twice the printed bound, floored at 2e-14, the FP64 rounding of the operator's entries
        assert dev_ <= max(2 * float(bound), 2e-14)
    assert ratio.min() >= -3.0
    assert abs(ev[5] - (-1.0 / 3.0)) < 1e-13
    core.close()


def test_table4_chapman_enskog_viscosity():
    """Hard spheres, K_max = 8, L = 2: f_mu^(K) = L_00 [(L_{kk'})_{k,k' <= K}^{-1}]_00 on the l = 2
    block of the GPU's linearized operator, against Table 4 (6 printed digits) and the exact
    K = 1 value 205/202."""
    Kmax, L = 8, 2
    core = wefq.Core("hs", Kmax, L, device=0, precisions=("fp64",))
    NK = Kmax + 1
    q = 2 * 2 + 2 + 0                                          # (l, m) = (2, 0)
    cols = q * NK + np.arange(NK)
    L2 = linearized(core, cols)[q * NK:(q + 1) * NK, :]        # rows (k1, 2, 0), columns (k, 2, 0)
    fmu = [L2[0, 0] * np.linalg.inv(L2[:K + 1, :K + 1])[0, 0] for K in range(Kmax + 1)]
    say("[table4] " + " ".join(f"{x:.7f}" for x in fmu))
    table = golden("table4_viscosity.txt")
    for K, val in table[:-1]:
        assert abs(fmu[int(K)] - float(val)) <= 5e-7
    assert abs(fmu[1] - 205 / 202) < 1e-12
    assert all(b > a for a, b in zip(fmu, fmu[1:]))
    assert 1.016028 < fmu[8] <= float(table[-1][1]) + 5e-7
    core.close()


def test_stress_relaxation_follows_linear_theory():
    """Section 5's transient stress relaxation, hard spheres, K = L = 8: a Maxwellian with a
    small (k, l, m) = (0, 2, 0) shear perturbation, RK4 in FP64 on the GPU.  The shear mode
    follows the linear prediction [exp(L_2 t)]_{00} from the GPU's own linearized operator to
    O(eps); energy cascades into the k > 0 modes of l = 2; the invariants stay exactly put."""
    from scipy.linalg import expm
    K = L = 8
    NK = K + 1
    core = wefq.Core("hs", K, L, device=0, precisions=("fp64",))
    q = 6                                                      # (l, m) = (2, 0)
    cols = q * NK + np.arange(NK)
    L2 = linearized(core, cols)[q * NK:(q + 1) * NK, :]
    eps, dt, n = 1e-4, 0.05, 60
    c0 = np.zeros((1, core.N))
    c0[0, 0] = 1.0
    c0[0, q * NK] = eps
    c = torch.tensor(c0, device=dev())
    inv = core.rk_integrate(c, dt, n, scheme="rk4", precision="fp64")
    got = c.cpu().numpy()[0]
    lin = eps * expm(L2 * (dt * n))[:, 0]                      # the whole l = 2, m = 0 block
    say(f"[stress] t={dt * n}: shear {got[q * NK] / eps:.6f} linear {lin[0] / eps:.6f}")
    assert inv == 0.0
    assert abs(got[q * NK] - lin[0]) < 1e-3 * eps              # nonlinear terms are O(eps^2)
    assert np.abs(got[q * NK:(q + 1) * NK] - lin).max() < 1e-3 * eps
    assert got[q * NK] < 0.9 * eps                             # it has decayed
    assert np.abs(got[q * NK + 1:(q + 1) * NK]).max() > 1e-3 * eps   # cascade into k > 0
    inv_idx = [0, 1, NK, 2 * NK, 3 * NK]
    assert np.array_equal(got[inv_idx], c0[0, inv_idx])
    core.close()
