"""The DOE kernels' patch transform on its own (rw_patch_dft) against numpy's
complex128 FFT of the zero-padded patch (Formalism: the local angular spectrum
of a P x P patch zero-padded to M x M), for every supported M, half and full
patches and a batch that is not a multiple of the grid."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rw():
    import paper_2605_15418_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pkg.load_library()
    return pkg


@pytest.mark.parametrize("M", [16, 32, 64])
@pytest.mark.parametrize("full", [False, True])
def test_patch_dft_matches_numpy(rw, M, full):
    P = M if full else M // 2
    rng = np.random.default_rng(M + int(full))
    n = 37
    x = (rng.normal(size=(n, P, P)) + 1j * rng.normal(size=(n, P, P))).astype(np.complex64)
    out = rw.patch_dft(torch.tensor(x, device="cuda"), M).cpu().numpy()
    xp = np.zeros((n, M, M), dtype=np.complex128)
    xp[:, :P, :P] = x
    ref = np.fft.fft2(xp)
    err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
    assert err < 2e-6, err


def test_patch_dft_rejects_unsupported_sizes(rw):
    x = torch.zeros((2, 8, 8), dtype=torch.complex64, device="cuda")
    with pytest.raises(rw.RWError):
        rw.patch_dft(x, 128)
    with pytest.raises(rw.RWError):
        rw.patch_dft(torch.zeros((2, 40, 40), dtype=torch.complex64, device="cuda"), 32)
