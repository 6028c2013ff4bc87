"""lq_schur_noalloc (the Schur operator with its odd intermediate in the
library's static device scratch, for callers that cannot allocate) against
lq_schur with a caller-supplied temporary, through the C ABI: two calls in a
row on lattices of decreasing size per precision and form, the second
smaller, both also within the FP64 oracle's tolerance; sizes beyond the
scratch array are refused with an error."""
import numpy as np
import pytest

from oracle import evenodd
from tests.gpu_common import TOL, case, rel, say

pytestmark = pytest.mark.gpu

KAPPA, CSW = 0.1350, 1.0


@pytest.fixture(scope="module")
def lq():
    from paper_1103_1363_amd import lq as _lq
    return _lq


def run_pair(lq, dims, prec, dagger):
    u, _, e, _ = case(dims, "smooth", 5)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    lat.set_clover(KAPPA, CSW)
    din = lat.to_device(e, lq.EVEN, prec)
    ref_out = lat.new_field(lq.EVEN, prec)
    tmp = lat.new_field(lq.ODD, prec)
    lat.schur(ref_out, din, tmp, dagger, prec)
    out = lat.new_field(lq.EVEN, prec)
    lat.schur_noalloc(out, din, dagger, prec)
    got = lat.to_host(out, lq.EVEN, prec)
    want = lat.to_host(ref_out, lq.EVEN, prec)
    oracle = evenodd.WilsonClover(u, KAPPA, CSW).schur(e, dagger=dagger)
    return got, want, oracle


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("dagger", [False, True])
def test_schur_noalloc_matches_schur(lq, prec, dagger):
    for dims in [(8, 8, 8, 16), (4, 4, 4, 6)]:  # second call on a smaller lattice
        say(f"schur_noalloc dims={dims} prec={prec} dagger={dagger}")
        got, want, oracle = run_pair(lq, dims, prec, dagger)
        # same kernels on the same inputs: identical results
        assert np.array_equal(got, want), rel(got, want)
        assert rel(got, oracle) <= TOL[prec]


def test_schur_noalloc_multiple_rhs(lq):
    dims = (4, 4, 4, 8)
    u, _, e, _ = case(dims, "smooth", 6)
    lat = lq.Lattice(dims)
    lat.upload_gauge(u)
    lat.set_clover(KAPPA, CSW)
    e2 = np.stack([e, 2.0 * e[::-1].copy()])
    din = lat.to_device(e2, lq.EVEN, lq.F32)
    out = lat.new_field(lq.EVEN, lq.F32, 2)
    lat.schur_noalloc(out, din, False, lq.F32, 2)
    got = lat.to_host(out, lq.EVEN, lq.F32, 2)
    wc = evenodd.WilsonClover(u, KAPPA, CSW)
    for r in range(2):
        assert rel(got[r], wc.schur(e2[r])) <= TOL[1]


def test_schur_noalloc_rejects_sizes_beyond_scratch(lq):
    """32^3x64: one odd FP64 field needs 201 MB, FP32 101 MB, both above the
    64 MiB scratch; FP16 (54.5 MB) fits.  F16X is refused (its tables are
    allocated by the library)."""
    dims = (32, 32, 32, 64)
    lat = lq.Lattice(dims)
    a = lat.new_field(lq.EVEN, lq.F16)
    b = lat.new_field(lq.EVEN, lq.F16)
    for prec in (lq.F64, lq.F32):
        with pytest.raises(lq.LQError, match="scratch"):
            lat.schur_noalloc(b, a, False, prec)
    with pytest.raises(lq.LQError, match="clover"):
        lat.schur_noalloc(b, a, False, lq.F16)  # fits, but no clover term yet
    with pytest.raises(lq.LQError, match="precision"):
        lat.schur_noalloc(b, a, False, lq.F16X)
