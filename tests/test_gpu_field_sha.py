"""Device building blocks against Python integers and hashlib (GPU)."""
import hashlib
import random

import numpy as np
import pytest
import torch

from tests._helpers import P, R_MONT, dev, ints_of, limbs_of

pytestmark = pytest.mark.gpu

EDGE = [0, 1, 2, P - 1, P - 2, (1 << 253), (1 << 254) % P, R_MONT % P, (R_MONT * R_MONT) % P,
        (P - 1) // 2, 0xFFFFFFFF, (1 << 232) - 1, P - (1 << 29)]


def _operands(seed, n):
    rng = random.Random(seed)
    a = [rng.randrange(P) for _ in range(n)] + [x for x in EDGE for _ in EDGE]
    b = [rng.randrange(P) for _ in range(n)] + [y for _ in EDGE for y in EDGE]
    return a, b


@pytest.fixture(scope="module")
def zc():
    from paper_2606_16146_amd import zc as z
    z.lib()
    return z


@pytest.mark.parametrize("op", [0, 1, 2])
def test_field_ops_match_python(zc, op):
    a, b = _operands(op, 4096)
    out = ints_of(zc.test_field(op, dev(limbs_of(a)), dev(limbs_of(b))))
    torch.cuda.synchronize()
    f = {0: lambda x, y: x * y % P, 1: lambda x, y: (x + y) % P, 2: lambda x, y: (x - y) % P}[op]
    assert out == [f(x, y) for x, y in zip(a, b)]


def test_montgomery_raw_on_lazy_inputs(zc):
    """Any 256-bit operands (up to ~5.3p): result is A*B*R^-1 mod p."""
    rng = random.Random(9)
    a = [rng.randrange(1 << 256) for _ in range(2048)] + [(1 << 256) - 1, 0, 5 * P, 5 * P + 7]
    b = [rng.randrange(1 << 256) for _ in range(2048)] + [(1 << 256) - 1, (1 << 256) - 1, 5 * P, 3]
    out = ints_of(zc.test_field(3, dev(limbs_of(a)), dev(limbs_of(b))))
    rinv = pow(R_MONT, -1, P)
    assert out == [x * y * rinv % P for x, y in zip(a, b)]


def test_mont_conversions(zc):
    a, _ = _operands(3, 1024)
    tm = ints_of(zc.test_field(4, dev(limbs_of(a)), dev(limbs_of(a))))
    assert tm == [x * R_MONT % P for x in a]
    big = a + [(1 << 256) - 1, 5 * P]
    fm = ints_of(zc.test_field(5, dev(limbs_of(big)), dev(limbs_of(big))))
    rinv = pow(R_MONT, -1, P)
    assert fm == [x * rinv % P for x in big]


def test_extension_bound_worst_case(zc):
    """e = a + 10 b built by plain additions (< 11p) squared: the largest product inputs."""
    a, b = _operands(4, 1024)
    a += [P - 1, P - 1, 0]
    b += [P - 1, 0, P - 1]
    out = ints_of(zc.test_field(6, dev(limbs_of(a)), dev(limbs_of(b))))
    rinv = pow(R_MONT, -1, P)
    assert out == [(x + 10 * y) ** 2 * rinv * rinv % P for x, y in zip(a, b)]


def test_sha256_all_lengths_match_hashlib(zc):
    rng = random.Random(11)
    lengths = list(range(0, 200)) + [244, 255, 256, 320, 352, 384, 416, 976, 1100]
    for n in lengths:
        msg = bytes(rng.randrange(256) for _ in range(n))
        padded = msg + bytes(-len(msg) % 4) + bytes(4)
        words = np.frombuffer(padded, dtype=np.uint32).copy()
        got = zc.test_sha256(dev(words), n).cpu().numpy().tobytes()
        assert got == hashlib.sha256(msg).digest(), n
