"""eg_rnorm_noalloc (static per-device workspace, no allocation, result in
device memory) against eg_rnorm on the same residuals, through the C ABI:
two calls in a row, the second on a smaller handle, each to 1e-13 of the
norm (both FP64; the two sum the squares in different orders)."""

import numpy as np
import pytest

from eg_inputs import ogrid, cubed_sphere_shell
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _case(mesh, p, seed):
    import paper_1807_01151_amd as P
    S = P.Solver(mesh, p)
    rng = np.random.default_rng(seed)
    r = to_dev(rng.standard_normal((mesh.n_elem, S.V, S.N(p))))
    return S, r


@pytest.mark.parametrize("first,second", [((ogrid(128, 64), 3), (ogrid(24, 12), 1)),
                                          ((cubed_sphere_shell(8, 8), 2), (cubed_sphere_shell(2, 2), 1))],
                         ids=["2d", "3d"])
def test_rnorm_noalloc_matches_rnorm(first, second):
    import torch
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    for k, (mesh, p) in enumerate((first, second)):
        print(f"call {k}: {mesh.name} p={p} elements={mesh.n_elem}", flush=True)
        S, r = _case(mesh, p, 70 + k)
        want = S.rnorm(r)
        S.rnorm_noalloc(r, out)
        torch.cuda.synchronize()
        got = float(out.cpu()[0])
        print(f"  noalloc {got:.17e} rnorm {want:.17e}", flush=True)
        assert abs(got - want) <= 1e-13 * want
        S.close()
