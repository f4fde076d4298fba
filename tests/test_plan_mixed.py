"""CPU checks of the mixed-radix stage lists the planner builds (no GPU): for
every pass that runs on the register mixed-radix kernels, the radices multiply
to the pass length, the register stages divide the points per thread Q (middle
stages may also take 2, 3, 4, 5 or 7), the first is Q, and the last is one the
kernels are instantiated for (Q itself, 2, 3 or the family's odd prime), or,
for the families with a gather form (Q = 7, 9, 12, 14, 15 and FP32 21), a radix
that does not divide Q when no prime of Q divides the rest; rows never take 20
points per thread, and the options that cap Q are honoured."""
import pytest

# (Q, last radix) pairs that have kernels, per dtype
PAIRS = {"f32": {(5, 5), (7, 7), (9, 9), (9, 3), (10, 10), (10, 2), (10, 5), (12, 12), (12, 2), (12, 3), (14, 14),
                 (14, 2), (14, 7), (15, 15), (15, 3), (15, 5), (20, 20), (20, 2), (20, 5), (21, 21), (21, 3),
                 (21, 7), (25, 25), (25, 5)},
         "f64": {(5, 5), (7, 7), (9, 9), (9, 3), (10, 10), (10, 2), (10, 5), (12, 12), (12, 2), (12, 3), (14, 14),
                 (14, 2), (14, 7), (15, 15), (15, 3), (15, 5)}}
GATHER = {"f32": {7, 9, 12, 14, 15, 21}, "f64": {7, 9, 12, 14, 15}}

SHAPES = [(8000, 8000), (4000, 4000), (2000, 1000), (250, 160), (96, 768), (75, 50), (20, 40, 100), (640,),
          (1536, 40), (400, 400, 400), (800, 800, 800), (192, 96), (96, 48), (250,), (20, 500), (1250, 3000),
          (625, 48), (3125,), (120, 360), (6300, 6720), (630, 420), (1470, 90), (210, 3360), (63, 105, 42),
          (49, 64), (35, 64), (42, 40), (210, 16), (27, 81), (54, 162), (343, 16), (63, 21), (175, 30),
          (189, 20), (105, 98), (30, 60), (243, 2), (3969, 16)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_mixed_stage_lists_are_valid(shape, dtype):
    import paper_2105_06676_amd as sfft
    for p in sfft.plan_describe(shape, dtype)["passes"]:
        q = p["mixed_q"]
        if not q:
            continue
        rad = p["radices"]
        prod = 1
        for x in rad:
            # register stages (first, last) divide Q; middle stages may take 2, 3, 4, 5, 7
            assert q % x == 0 or x in (2, 3, 4, 5, 7), (shape, p)
            prod *= x
        assert prod == p["L"], (shape, p)
        assert rad[0] == q and len(rad) >= 2, (shape, p)
        if q % rad[-1]:
            # gather form: no prime of Q divides the length beyond the first stage
            assert q in GATHER[dtype], (shape, p)
            rest = p["L"] // q
            assert all(rest % f for f in (2, 3, 5, 7) if q % f == 0), (shape, p)
        else:
            assert (q, rad[-1]) in PAIRS[dtype], (shape, p)
        if p["kind"] == "row":
            assert q != 20, (shape, p)  # no 20-point row kernels


def test_mixed_q_options_cap_points_per_thread():
    import paper_2105_06676_amd as sfft
    try:
        sfft.set_option("mixed_col_q", 10)
        for p in sfft.plan_describe((400, 400, 400), "f32")["passes"]:
            if p["kind"] == "col" and p["mixed_q"]:
                assert p["mixed_q"] <= 10
        sfft.set_option("mixed_row_q", 5)
        for p in sfft.plan_describe((8000, 8000), "f32")["passes"]:
            if p["kind"] == "row" and p["mixed_q"]:
                assert p["mixed_q"] == 5
    finally:
        sfft.set_option("mixed_col_q", 0)
        sfft.set_option("mixed_row_q", 0)
    with pytest.raises(sfft.SfftError):
        sfft.set_option("mixed_row_q", 7)


def _strided_levels(shape, dtype):
    import paper_2105_06676_amd as sfft
    d = sfft.plan_describe(shape, dtype)
    return [p for p in d["passes"] if p["kind"] == "col"], d["levels"]


def _register(p):
    return bool(p["fast"] or p["mixed_q"])


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("shape", [(600, 4096), (640, 4096), (720, 4096), (768, 4096), (1024, 4096),
                                   (640, 200, 256), (256, 768, 64)])
def test_strided_axis_up_to_1024_in_one_register_pass(shape, dtype):
    """One pass over an axis the register kernels cover whole (every split moves the
    spectrum through HBM twice more)."""
    cols, _ = _strided_levels(shape, dtype)
    axes = len(shape) - 1  # strided axes: forward and inverse passes, one fused middle pass
    assert len(cols) == 2 * axes - 1, (shape, cols)
    assert all(_register(p) for p in cols), (shape, cols)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n", [1200, 1280, 1500, 1536, 1600, 8000, 6300, 960])
def test_split_levels_run_on_register_kernels(n, dtype):
    """Axes split into two levels put both on the register kernels and never leave a
    level of fewer than 16 points behind a large power-of-two factor (1536 once went
    512 x 3, the 3-point level on the generic kernels)."""
    cols, _ = _strided_levels((n, 64), dtype)
    assert len(cols) == 3, cols
    assert all(_register(p) for p in cols), (n, cols)
    assert all(p["L"] >= 16 for p in cols), (n, cols)


def test_power_of_two_level_placement():
    """FP32 runs the power-of-two level in the fused middle pass, FP64 first."""
    c32, _ = _strided_levels((8000, 8000), "f32")
    c64, _ = _strided_levels((8000, 8000), "f64")
    assert [p["L"] for p in c32] == [125, 64, 125]
    assert [p["L"] for p in c64] == [64, 125, 64]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("L", [49, 343, 27, 81, 243, 54, 162, 35, 42, 70, 105, 175, 210, 30, 60, 63, 189, 245])
def test_lengths_mixing_primes_take_register_columns(L, dtype):
    """Strided lengths such as 7^b, 3^b, 2 3^b and those whose factors share no
    prime with any Q (35, 42, 210, ...) run on the register kernels."""
    cols, _ = _strided_levels((L, 64), dtype)
    assert len(cols) == 1 and cols[0]["mixed_q"], (L, cols)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("shape", [(64, 125), (30, 49), (20, 27), (12, 105), (125,), (343,), (945,), (10, 12, 35)])
def test_odd_real_rows_take_register_kernels(shape, dtype):
    """Odd last extents: the rows are n-point complex transforms on the register
    kernels (odd points per thread), not the generic ones."""
    import paper_2105_06676_amd as sfft
    rows = [p for p in sfft.plan_describe(shape, dtype)["passes"] if p["kind"] == "row"]
    assert rows and all(p["mixed_q"] % 2 == 1 for p in rows), (shape, rows)
    assert all(p["L"] == shape[-1] for p in rows), (shape, rows)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n", [100000, 40000, 18522, 1000000])
def test_long_1d_complex_middle_rows_take_register_kernels(n, dtype):
    import paper_2105_06676_amd as sfft
    mids = [p for p in sfft.plan_describe((n,), dtype)["passes"] if p["kind"] == "row"]
    assert len(mids) == 1 and mids[0]["mixed_q"], (n, mids)
