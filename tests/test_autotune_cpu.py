"""The autotuner's choice rule, on made-up timings (CPU)."""
import pytest


@pytest.mark.parametrize("storage,model,default", [("f32", 0, (8, 1)), ("f16", 0, (16, 1)), ("f16", 1, (8, 1)),
                                                   ("f32", 1, (8, 1))])
def test_default_shape_kept_within_the_margin_and_left_beyond_it(storage, model, default):
    from paper_2009_12584_amd import autotune as T

    d = T.default_shape(storage, model)
    assert d == default and d in T.CANDIDATES
    other = next(c for c in T.CANDIDATES if c != d)
    near = {c: 100.0 for c in T.CANDIDATES}
    near[other] = 100.0 * (1 - T.MARGIN / 2)  # faster, but within the margin
    assert T.pick(near, storage, model) == d
    far = dict(near)
    far[other] = 100.0 * (1 - 2 * T.MARGIN)
    assert T.pick(far, storage, model) == other
    slower = {c: 100.0 + (0 if c == d else 1 + i) for i, c in enumerate(T.CANDIDATES)}
    assert T.pick(slower, storage, model) == d
