"""The autotuner's choice rule, on made-up timings (CPU)."""


def test_default_shape_kept_within_the_margin_and_left_beyond_it():
    from paper_2009_12584_amd import autotune as T

    d = T.CANDIDATES[0]
    other = T.CANDIDATES[1]
    near = {c: 100.0 for c in T.CANDIDATES}
    near[other] = 100.0 * (1 - T.MARGIN / 2)  # faster, but within the margin
    assert T.pick(near) == d
    far = dict(near)
    far[other] = 100.0 * (1 - 2 * T.MARGIN)
    assert T.pick(far) == other
    slower = {c: 100.0 + i for i, c in enumerate(T.CANDIDATES)}
    assert T.pick(slower) == d
