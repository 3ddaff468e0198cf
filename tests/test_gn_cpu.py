"""Host-side pieces of the Gauss-Newton driver (Section 4.5), no GPU.

* The roughness operator R (first differences between face-adjacent cells)
  equals an explicit sparse matrix built cell pair by cell pair, and
  roughness_T is its transpose (<R p, z> = <p, R^T z>), in 2-D and 3-D.
* The data weights are the inverse standard deviation of an absolute floor
  and a relative term in quadrature.
"""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")
gn = pytest.importorskip("paper_2609_14982_amd.gn")


def _explicit_R(cells):
    c0, c1, c2 = cells
    idx = lambda i, j, k: i + c0 * (j + c1 * k)  # noqa: E731
    rows, cols, vals, r = [], [], [], 0
    for di, dj, dk in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
        if (di and c0 == 1) or (dj and c1 == 1) or (dk and c2 == 1):
            continue
        for k in range(c2 - dk):
            for j in range(c1 - dj):
                for i in range(c0 - di):
                    rows += [r, r]
                    cols += [idx(i + di, j + dj, k + dk), idx(i, j, k)]
                    vals += [1.0, -1.0]
                    r += 1
    return sp.csr_matrix((vals, (rows, cols)), shape=(r, c0 * c1 * c2))


@pytest.mark.parametrize("cells", [(7, 5, 1), (5, 4, 3)], ids=["2d", "3d"])
def test_roughness_is_the_difference_matrix(cells):
    Rx = _explicit_R(cells)
    rng = np.random.default_rng(3)
    p = rng.standard_normal(Rx.shape[1])
    z = rng.standard_normal(Rx.shape[0])
    Rp = gn.roughness(torch.from_numpy(p), cells).numpy()
    RTz = gn.roughness_T(torch.from_numpy(z), cells).numpy()
    assert np.allclose(Rp, Rx @ p, rtol=0, atol=1e-14)
    assert np.allclose(RTz, Rx.T @ z, rtol=0, atol=1e-13)
    assert abs(Rp @ z - p @ RTz) <= 1e-12 * np.abs(Rp @ z)


def test_data_weights():
    d = np.array([0.0, 1.0, 2.0])
    w = gn.data_weights(d, 3e-4, 3e-3)
    assert np.allclose(w, 1.0 / np.sqrt(9e-8 + (3e-3 * d) ** 2), rtol=1e-15)
