"""Labels of the learned (q, p) selector on the GPU against the FP64 oracle.

The training labels come from batched GPU solves (one batch per class, the
matrix's own Omega stream) and exact residual norms computed from the planted
factors by a Krylov iteration.  Here the same machinery runs on 288 small
generated matrices stored in f64 (f64 arithmetic, so the two sides differ by
rounding only) and is compared with oracle.learned, which runs the FP64
oracle rSVD for every class and takes the residual's 2-norm by a dense SVD:

* excess errors agree class by class to 1e-8 (absolute);
* every "within 1 %" decision agrees outside a band of +-0.1 % around the
  target (inside it rounding may decide either way);
* labels agree for every matrix none of whose class errors lies in that band.
"""
import numpy as np
import pytest
import torch

from oracle import learned as lrn

pytestmark = pytest.mark.gpu
COUNT = 288


def test_gpu_labels_match_oracle():
    from paper_1608_02148_amd import learned as L
    from synth import learned_data as ld
    data = ld.build(COUNT, 4242, device="cuda", out_dtype=torch.float64, m_range=(60, 300),
                    n_range=(40, 160), k_max=20)
    ks = [int(x) for x in data["spec"]["k"]]
    tab = L.excess_table(data, precision="plain", seed=2148)
    lab, ok = L.labels_from_table(tab, ks)

    band = 0.001
    compared = 0
    ora_tab = np.zeros_like(tab)
    for b in range(COUNT):
        A = data["A"][b].cpu().numpy()
        k = ks[b]
        sn = float(data["sigma"][b][k])
        for c in range(lrn.N_CLASSES):
            q, p = lrn.class_pair(c)
            ora_tab[b, c] = lrn.excess_error(A, k, q, p, seed=2148, stream_id=b, sigma_next=sn)
        want, reach = lrn.label(A, k, seed=2148, stream_id=b, sigma_next=sn)
        if np.all(np.abs(ora_tab[b] - 0.01) > band):
            compared += 1
            assert lab[b] == want and ok[b] == reach, (b, lab[b], want, tab[b], ora_tab[b])
    np.testing.assert_allclose(tab, ora_tab, rtol=0, atol=1e-8)
    outside = np.abs(ora_tab - 0.01) > band
    assert np.array_equal((tab <= 0.01)[outside], (ora_tab <= 0.01)[outside])
    assert compared >= 256, compared
    print(f"labels compared on {compared} of {COUNT} matrices, all equal")
