"""The GPU's normals against the oracle's, counter by counter: Philox4x32-10
and the Box-Muller map are specified once (Random123's generator, uniforms
(x + 1/2) 2^-32, pairs sqrt(-2 ln u_a) (cos, sin)(2 pi u_b)) and implemented
independently on both sides.  The Philox outputs must agree exactly; the
normals to the rounding of the two evaluations:

* FP64: the oracle forms the angle 2 pi u_b in FP64 before cos/sin, an
  absolute angle error up to 2^-51 (half an ulp of a number below 8), which
  the radius r <= 6.7 scales to ~13 ulp of 1 for |z| <= 1, and to at most
  2^-51 / |cos| <= 13 ulp relative for |z| >= 1 (then |cos| >= 1/6.7); the
  GPU's own functions are within ~1 ulp.  Bar: 24 ulp of max(|z|, 1).
* FP32: the uniform is formed in FP32, so near u = 1 the gap 1 - u carries
  an absolute rounding of up to 2^-25, which moves the small radius
  r = sqrt(2 (1 - u)) by up to 2^-25 / r: absolute, and only for tiny |z|.
  Bar: 2e-4 of max(|z|, 1), and 1e-6 relative where r > 0.5."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

CASES = [(1234, 0, 0), (1234, 7, 1), (2 ** 40 + 99, 123456, 2), (0, 4294967295, 0)]


def _oracle(seed, step, tag, site0, n, slots):
    out = np.zeros((n, slots))
    for i in range(n):
        for s in range(slots):
            out[i, s] = O.normal(seed, site0 + i, step, tag, s)
    return out


@pytest.mark.parametrize("seed,step,tag", CASES)
def test_normals_match_oracle(seed, step, tag):
    from paper_1104_0078_amd import lbl
    n, slots = 3000, 16
    for site0 in (0, 2 ** 31 - 1000):
        ref = _oracle(seed, step, tag, site0, n, slots)
        g64 = lbl.diag_normals(lbl.LBL_FP64, seed, step, tag, site0, n, slots)
        g32 = lbl.diag_normals(lbl.LBL_FP32DEV, seed, step, tag, site0, n, slots)
        e64 = np.abs(g64 - ref) / np.maximum(np.abs(ref), 1.0)
        e32 = np.abs(g32 - ref) / np.maximum(np.abs(ref), 1.0)
        # radius of each pair: sqrt(z_even^2 + z_odd^2)
        rr = np.sqrt(ref[:, 0::2] ** 2 + ref[:, 1::2] ** 2).repeat(2, axis=1)
        big = rr > 0.5
        e32b = (np.abs(g32 - ref)[big] / np.maximum(np.abs(ref[big]), 1e-300 + rr[big]))
        print("seed %d step %d tag %d site0 %d: FP64 %.1f ulp (at |z| %.3g); FP32 %.2e "
              "(at r %.3g), %.2e where r > 0.5"
              % (seed, step, tag, site0, e64.max() / 2 ** -52, abs(ref.flat[e64.argmax()]),
                 e32.max(), rr.flat[e32.argmax()], e32b.max()), flush=True)
        assert e64.max() <= 24 * 2 ** -52
        assert e32.max() <= 2e-4
        assert e32b.max() <= 1e-6
