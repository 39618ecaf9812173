"""The plain 3-D transforms (fm_fft_forward / fm_fft_backward) against the oracle's: the
forward spectrum element by element (half spectrum on the real-to-complex axis), the
backward transform of the oracle's spectrum, and the round trip prod(n_log) * f, in both
precisions, for periodic grids (the transform pair of the paper's FFT comparison) and for
mixed boundary conditions."""
import numpy as np
import pytest

import oracle as O
import paper_2211_07777_amd as F

from gpu_common import TOL32, TOL64, check_conventions, rel_linf

pytestmark = pytest.mark.gpu

CASES = [
    ([32, 24, 20], [[2, 2]] * 3, F.CELL),
    ([16, 12, 10], [[2, 2]] * 3, F.NODE),
    ([10, 12, 9], [[3, 3], [0, 1], [2, 2]], F.CELL),
    ([7, 9, 12], [[1, 3], [0, 0], [3, 3]], F.NODE),
    ([8, 6, 10], [[0, 0], [1, 1], [2, 2]], F.CELL),   # the only DFT axis is the last one
    ([6, 7, 5], [[0, 1], [1, 0], [1, 1]], F.NODE),    # symmetric axes only
    ([5, 8, 6], [[3, 0], [2, 2], [3, 3]], F.CELL),
]


def _oracle_spectrum(plan, f, n, h, bc, layout):
    dims, axes, _, _ = plan.spectrum_layout()
    full = O.forward(f, n, h, bc, layout)                     # [sz][sy][sx]
    perm = np.transpose(full, [2 - a for a in axes])          # slow -> fast as the plan
    return full, perm[:dims[0], :dims[1], :dims[2]]


@pytest.mark.parametrize("prec,tol", [(F.F64, TOL64), (F.F32, TOL32)])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_forward_backward_against_oracle(case, prec, tol):
    import torch
    n, bc, layout = CASES[case]
    h = [0.1, 0.12, 0.09]
    plan = F.Plan(n, h, bc, layout, F.CHAT2, prec)
    f = np.random.default_rng(case).standard_normal(O.user_shape(n, layout))
    x = torch.from_numpy(f).to("cuda", plan.dtype)
    spec = plan.fft_forward(x)
    torch.cuda.synchronize()
    full, ref = _oracle_spectrum(plan, f, n, h, bc, layout)
    got = spec.cpu().numpy().astype(np.complex128 if spec.is_complex() else np.float64)
    if not spec.is_complex():
        assert np.abs(ref.imag).max() == 0.0
        ref = ref.real
    assert got.shape == ref.shape
    assert rel_linf(got, ref) < tol, ("forward", n, bc, layout)
    # backward of the oracle's spectrum
    spec_in = torch.from_numpy(np.ascontiguousarray(ref)).to("cuda", spec.dtype)
    u = plan.fft_backward(spec_in)
    torch.cuda.synchronize()
    u = u.double().cpu().numpy()
    check_conventions(u, bc, layout)
    assert rel_linf(u, O.backward(full, n, h, bc, layout)) < tol, ("backward", n, bc, layout)
    # round trip on the device
    v = plan.fft_backward(plan.fft_forward(x))
    torch.cuda.synchronize()
    nlog = np.prod([O.axis_info(n[a], h[a], layout, *bc[a])["nlog"] for a in range(3)])
    assert rel_linf(v.double().cpu().numpy(), O.backward(O.forward(f, n, h, bc, layout), n, h, bc, layout)) < tol
    assert np.isclose(np.abs(O.backward(O.forward(f, n, h, bc, layout), n, h, bc, layout)).max(),
                      nlog * np.abs(f).max(), rtol=0.5)  # sanity: unnormalised pair
    plan.close()


def test_several_components_and_explicit_workspace():
    import torch
    n, bc, layout = [12, 10, 8], [[2, 2], [3, 3], [3, 3]], F.CELL
    h = [0.1, 0.1, 0.1]
    plan = F.Plan(n, h, bc, layout, F.CHAT2, F.F64, F.POISSON, ncomp=2)
    f = np.random.default_rng(9).standard_normal((2,) + O.user_shape(n, layout))
    x = torch.from_numpy(f).cuda()
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    spec = plan.fft_forward(x, workspace=ws)
    torch.cuda.synchronize()
    for c in range(2):
        _, ref = _oracle_spectrum(plan, f[c], n, h, bc, layout)
        assert rel_linf(spec[c].cpu().numpy(), ref) < TOL64
    y = plan.fft_backward(spec, workspace=ws)
    torch.cuda.synchronize()
    for c in range(2):
        full = O.forward(f[c], n, h, bc, layout)
        assert rel_linf(y[c].cpu().numpy(), O.backward(full, n, h, bc, layout)) < TOL64
    plan.close()
