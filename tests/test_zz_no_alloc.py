"""The allocation-free time-step control (te_timestep_noalloc) against
te_timestep through the C ABI: identical decisions, next steps and largest
changes on two calls in a row, the second on a smaller input, and its
argument errors."""
import ctypes as C

import numpy as np
import pytest

from tests.gpu_util import dev, say, torch_cuda

pytestmark = pytest.mark.gpu


def _call(fn, a, b, n, dt, dT_max, eps, stream):
    dn, acc, mc = C.c_double(0.0), C.c_int32(0), C.c_double(0.0)
    code = fn(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), n, dt, dT_max, eps, C.byref(dn), C.byref(acc),
              C.byref(mc), stream)
    return code, acc.value, dn.value, mc.value


def test_noalloc_timestep_equals_allocating_one():
    torch = torch_cuda()
    import paper_1804_10060_amd as te
    from paper_1804_10060_amd import _lib
    lib = _lib.load()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rng = np.random.default_rng(7)
    # first call: 3.1M entries (1024 partials, grid-stride), the second 1000
    # entries (4 partials): the second must not see the first's partials
    for n, dT_max, scale in ((3_100_017, 10.0, 4.0), (1000, 10.0, 30.0), (1000, 10.0, 0.5), (1, 1.0, 2.0)):
        say("noalloc timestep n =", n, "scale", scale)
        T_old = rng.uniform(290.0, 310.0, n)
        T_new = T_old + scale * rng.standard_normal(n)
        a, b = dev(T_new, torch.float64), dev(T_old, torch.float64)
        r1 = _call(lib.te_timestep, a, b, n, 2.5, dT_max, 0.9, stream)
        r2 = _call(lib.te_timestep_noalloc, a, b, n, 2.5, dT_max, 0.9, stream)
        assert r1[0] == 0 and r2[0] == 0
        assert r1 == r2, (r1, r2)
        assert r2[3] == float(np.max(np.abs(T_new - T_old)))   # max is exact
        # the Python binding routes to the same entry point
        assert te.timestep(a, b, 2.5, dT_max, 0.9, noalloc=True) == (bool(r1[1]), r1[2], r1[3])
    # no change doubles the step; n = 0 too
    z = dev(np.full(5000, 300.0), torch.float64)
    assert _call(lib.te_timestep_noalloc, z, z, 5000, 1.0, 10.0, 0.9, stream)[1:] == (1, 2.0, 0.0)
    assert _call(lib.te_timestep_noalloc, z, z, 0, 1.0, 10.0, 0.9, stream)[1:] == (1, 2.0, 0.0)
    # argument errors and a NaN, decided on the host or read back from the device
    assert _call(lib.te_timestep_noalloc, z, z, -1, 1.0, 10.0, 0.9, stream)[0] == _lib.TE_EINVAL
    assert _call(lib.te_timestep_noalloc, z, z, 10, 0.0, 10.0, 0.9, stream)[0] == _lib.TE_EINVAL
    assert _call(lib.te_timestep_noalloc, z, z, 10, 1.0, 10.0, 1.5, stream)[0] == _lib.TE_EINVAL
    zn = z.clone()
    zn[4321] = float("nan")
    assert _call(lib.te_timestep_noalloc, zn, z, 5000, 1.0, 10.0, 0.9, stream)[0] == _lib.TE_ENAN
    # after the error the next call is whole again
    assert _call(lib.te_timestep_noalloc, z, z, 5000, 1.0, 10.0, 0.9, stream)[1:] == (1, 2.0, 0.0)
