"""The kernels' elementary device arithmetic, function by function, in each kernel unit (the
single-job unit with literal series constants, the deferred-launch unit reading them from LDS,
the batched unit holding them in scalar registers), through tests/device_arith.hip:

* the divisions with bounded operands (kdiv) equal the correctly rounded quotient -- the
  compiler's FP64 division on the device and the host's IEEE division -- bit for bit, over the
  logarithm's atanh argument and two bands of exponents;
* the square root without argument scaling (ksqrt_n) equals the correctly rounded root for 0,
  +inf and every normal argument from 2^-1000 up, and for the kernels' own kinds of argument
  (1 - mu^2, -2 ln u);
* ln and sin/cos (FP64) equal the oracle's written-out series bit for bit over the whole range
  of finite doubles, around the reduction's multiples of pi/4 and at the special values;
* Philox4x32-10, the 53-bit uniform of two words and the SplitMix64 finaliser equal the
  oracle's (which its CPU tests pin against rocRAND and pybind11's finaliser);
* FP32 state: ln and sin/cos from the hardware's single-precision functions stay within 4e-7
  (ln: absolute, plus relative to |ln x|) and 2e-6 (sin/cos on |x| <= 2 pi) of FP64."""
import numpy as np
import pytest

import device_arith as D

pytestmark = pytest.mark.gpu

UNITS = ("single", "drain", "batched")
SQRT_HALF = 0.70710678118654757
SQRT2 = 1.4142135623730951


def f64_from(exp, rng, signed=True):
    """Doubles 2^exp x (1 + 52 random mantissa bits), random signs if `signed`."""
    exp = np.asarray(exp, dtype=np.int64)
    bits = ((exp + 1023).astype(np.uint64) << np.uint64(52)) | rng.integers(0, 1 << 52, exp.shape[0], dtype=np.uint64)
    if signed:
        bits |= rng.integers(0, 2, exp.shape[0], dtype=np.uint64) << np.uint64(63)
    return bits.view(np.float64)


def same_bits(got, ref):
    """Element-wise: identical bit patterns, or both NaN."""
    g, r = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    return (g.view(np.uint64) == r.view(np.uint64)) | (np.isnan(g) & np.isnan(r))


def assert_same(name, x, got, ref, y=None):
    ok = same_bits(got, ref)
    if not ok.all():
        i = np.nonzero(~ok)[0][:5]
        pairs = [(float(x[k]), None if y is None else float(y[k]), float(got[k]), float(ref[k])) for k in i]
        raise AssertionError(f"{name}: {int((~ok).sum())} of {ok.size} differ, first (x, y, got, ref): {pairs}")


def division_operands(rng):
    out = {}
    # the logarithm's atanh argument: f = m - 1 over m + 1 for the reduced mantissa m in
    # [sqrt(1/2), sqrt(2)) (f in (-0.30, 0.42], m + 1 in [1.7, 2.5))
    m = rng.uniform(SQRT_HALF, SQRT2, 1 << 22)
    m[:4] = [SQRT_HALF, 1.0, np.nextafter(SQRT2, 0.0), np.nextafter(1.0, 0.0)]
    out["ln atanh argument"] = (m - 1.0, m + 1.0)
    # a band of moderate exponents (paths over speeds, reciprocals of speeds and norms), with zeros
    n = 1 << 22
    a = f64_from(rng.integers(-400, 401, n), rng)
    a[:64] = 0.0
    out["exponents -400..400"] = (a, f64_from(rng.integers(-400, 401, n), rng))
    # a wider band: operands and quotient with exponents in -900..900 (3/4 of the draws kept)
    n = 1 << 24
    ea, eb = rng.integers(-900, 901, n), rng.integers(-900, 901, n)
    keep = np.abs(ea - eb) <= 899
    out["exponents -900..900"] = (f64_from(ea[keep], rng), f64_from(eb[keep], rng))
    return out


@pytest.mark.parametrize("unit", UNITS)
def test_bounded_division_is_correctly_rounded(unit):
    rng = np.random.default_rng(20250313)
    total = 0
    for name, (a, b) in division_operands(rng).items():
        print(f"{unit}: kdiv, {name}, {a.size} pairs", flush=True)
        q, q_ieee = D.apply(unit, D.DIV64, a, b, out1=True)
        ref = a / b
        assert_same(f"{unit} compiler division, {name}", a, q_ieee, ref, b)
        assert_same(f"{unit} kdiv, {name}", a, q, ref, b)
        total += a.size
    assert total > 2.0e7


@pytest.mark.parametrize("unit", UNITS)
def test_unscaled_square_root_is_correctly_rounded(unit):
    rng = np.random.default_rng(7)
    x = np.abs(f64_from(rng.integers(-1000, 1024, 1 << 23), rng, signed=False))
    # the kernels' arguments: 1 - mu^2 for mu on the 2^-52 grid, -2 ln u for u on the 2^-53 grid
    mu = rng.integers(-(1 << 52), (1 << 52) + 1, 1 << 20).astype(np.float64) * 2.0 ** -52
    u = (rng.integers(0, 1 << 53, 1 << 20, dtype=np.int64).astype(np.float64) + 1.0) * 2.0 ** -53
    x = np.concatenate([x, 1.0 - mu * mu, -2.0 * np.log(u),
                        [0.0, -0.0, np.inf, 2.0 ** -1000, 1.0, np.finfo(np.float64).max]])
    print(f"{unit}: ksqrt_n, {x.size} arguments", flush=True)
    r, r_ieee = D.apply(unit, D.SQRT64, x, out1=True)
    ref = np.sqrt(x)
    assert_same(f"{unit} compiler sqrt", x, r_ieee, ref)
    assert_same(f"{unit} ksqrt_n", x, r, ref)


def log_arguments(rng):
    tiny = np.finfo(np.float64).tiny
    return np.concatenate([
        np.abs(f64_from(rng.integers(-1022, 1024, 1 << 16), rng, signed=False)),
        1.0 + rng.uniform(-2.0 ** -10, 2.0 ** -10, 1 << 14),
        (rng.integers(0, 1 << 53, 1 << 14, dtype=np.int64).astype(np.float64) + 1.0) * 2.0 ** -53,
        10.0 ** rng.uniform(-3.0, 7.0, 1 << 14),
        rng.uniform(0.0, tiny, 256),                                    # subnormal
        [0.0, -0.0, -1.0, np.inf, -np.inf, np.nan, 5e-324, tiny, np.finfo(np.float64).max,
         1.0, np.nextafter(1.0, 0.0), np.nextafter(1.0, 2.0), SQRT_HALF, np.nextafter(SQRT_HALF, 0.0)],
    ])


@pytest.fixture(scope="module")
def log_case(oracle_lib):
    x = log_arguments(np.random.default_rng(11))
    return x, np.array([oracle_lib.log(float(v)) for v in x])


@pytest.mark.parametrize("unit", UNITS)
def test_log_equals_oracle(unit, log_case):
    x, ref = log_case
    print(f"{unit}: klog, {x.size} arguments", flush=True)
    got = D.apply(unit, D.LOG64, x)
    assert_same(f"{unit} klog", x, got, ref)
    # and within 2 ulp of the host's libm wherever the result is finite
    fin = np.isfinite(ref)
    libm = np.log(x[fin])
    assert (np.abs(got[fin] - libm) <= 2.0 * np.spacing(np.abs(libm))).all()


def sincos_arguments(rng):
    n = 1 << 16
    k = np.arange(-2000, 2001, dtype=np.float64)
    near = k * (np.pi / 4.0)
    return np.concatenate([
        10.0 ** rng.uniform(-12.0, 12.0, n) * rng.choice([-1.0, 1.0], n),
        rng.uniform(0.0, 1.0e5, 1 << 14),                                 # guiding-centre phases
        rng.uniform(0.0, 2.0 * np.pi, 1 << 14),                           # azimuths
        near, np.nextafter(near, np.inf), np.nextafter(near, -np.inf),
        [0.0, -0.0, np.inf, -np.inf, np.nan, 2.0e8, np.nextafter(2.0e8, 0.0), 1.0e15, -1.0e15,
         np.pi / 4.0, np.nextafter(np.pi / 4.0, 1.0)],
    ])


@pytest.fixture(scope="module")
def sincos_case(oracle_lib):
    x = sincos_arguments(np.random.default_rng(13))
    return x, np.array([oracle_lib.sincos(float(v)) for v in x])


@pytest.mark.parametrize("unit", UNITS)
def test_sincos_equals_oracle(unit, sincos_case):
    x, ref = sincos_case
    print(f"{unit}: ksincos, {x.size} arguments", flush=True)
    s, c = D.apply(unit, D.SINCOS64, x, out1=True)
    assert_same(f"{unit} sin", x, s, ref[:, 0])
    assert_same(f"{unit} cos", x, c, ref[:, 1])
    small = np.isfinite(x) & (np.abs(x) < 1.0e5)
    assert float(np.abs(s[small] - np.sin(x[small])).max()) < 1e-15
    assert float(np.abs(c[small] - np.cos(x[small])).max()) < 1e-15


@pytest.mark.parametrize("unit", UNITS)
def test_random_number_primitives_equal_oracle(unit, oracle_lib):
    rng = np.random.default_rng(17)
    w = rng.integers(0, 1 << 32, (4096, 6), dtype=np.uint64).astype(np.uint32)
    w[0] = 0
    w[1] = 0xFFFFFFFF
    got = D.apply(unit, D.PHILOX, w, out0_dtype=np.uint32, out0_width=4)
    ref = np.array([oracle_lib.philox(*(int(v) for v in row)) for row in w], dtype=np.uint32)
    np.testing.assert_array_equal(got, ref)
    ab = rng.integers(0, 1 << 32, (4096, 2), dtype=np.uint64).astype(np.uint32)
    ab[0] = 0
    ab[1] = 0xFFFFFFFF
    got = D.apply(unit, D.U53, ab)
    ref = np.array([oracle_lib.u53(int(a), int(b)) for a, b in ab])
    assert_same(f"{unit} uniform", ab[:, 0], got, ref)
    assert got.min() >= 0.0 and got.max() < 1.0
    z = rng.integers(0, 1 << 63, 4096, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, 4096, dtype=np.uint64)
    z[:2] = [0, 0xFFFFFFFFFFFFFFFF]
    got = D.apply(unit, D.MIX64, z, out0_dtype=np.uint64)
    ref = np.array([oracle_lib.lib().ko_mix64(int(v)) for v in z], dtype=np.uint64)
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("unit", UNITS)
def test_fp32_log_and_sincos_bounds(unit):
    rng = np.random.default_rng(19)
    x = np.concatenate([10.0 ** rng.uniform(-30.0, 30.0, 1 << 18),
                        (rng.integers(1, 1 << 24, 1 << 16) * 2.0 ** -24),
                        1.0 + rng.uniform(-1e-3, 1e-3, 1 << 14)]).astype(np.float32)
    got = D.apply(unit, D.LOG32, x, out0_dtype=np.float32).astype(np.float64)
    ref = np.log(x.astype(np.float64))
    err = np.abs(got - ref)
    bound = 4e-7 + 4e-7 * np.abs(ref)
    assert (err <= bound).all(), f"{unit} FP32 ln: worst {float((err / bound).max()):.2f} x bound"
    t = rng.uniform(-2.0 * np.pi, 2.0 * np.pi, 1 << 18).astype(np.float32)
    s, c = D.apply(unit, D.SINCOS32, t, out0_dtype=np.float32, out1=True)
    t64 = t.astype(np.float64)
    assert float(np.abs(s - np.sin(t64)).max()) <= 2e-6
    assert float(np.abs(c - np.cos(t64)).max()) <= 2e-6
