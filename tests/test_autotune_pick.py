"""Choice among measured decode options (host logic of the autotuner)."""
from paper_2602_12314_amd import autotune as AT


def _times(**ms):
    return {k.replace("_", "/splits="): v for k, v in ms.items()}


def test_rule_split_wins_within_tolerance():
    cands = AT.decode_candidates(shapes=("px64",), splits=(0, 16, 32))
    t = _times(px64_0=7.959, px64_16=7.956, px64_32=7.941)
    assert AT.pick_decode_options(cands, t) == {"decode_shape": "px64", "decode_splits": 0}


def test_clearly_faster_split_wins():
    cands = AT.decode_candidates(shapes=("px64",), splits=(0, 16))
    t = _times(px64_0=8.0, px64_16=7.5)
    assert AT.pick_decode_options(cands, t) == {"decode_shape": "px64", "decode_splits": 16}


def test_shape_choice_is_unaffected():
    cands = AT.decode_candidates(shapes=("px32", "px64"), splits=(0, 128))
    # px64 with the rule is 3 % slower than px32 with 128 splits: not a tie
    t = _times(px32_0=6.3, px32_128=6.0, px64_0=6.18, px64_128=6.25)
    assert AT.pick_decode_options(cands, t) == {"decode_shape": "px32", "decode_splits": 128}
    # within the tolerance the fastest rule candidate is taken, whatever its shape
    t = _times(px32_0=6.1, px32_128=6.0, px64_0=6.05, px64_128=6.2)
    assert AT.pick_decode_options(cands, t) == {"decode_shape": "px64", "decode_splits": 0}
