"""The DPP row operations that the k-NN and clip kernels compose into lane
moves inside a group, modelled from their definitions (a 64-lane wave in
rows of 16 lanes, each row in quads): every composition used must be the
exact lane map it stands for, in every group of the wave."""
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
CSRC = ROOT / "paper_2412_04514_amd" / "csrc"
WAVE = 64


def dpp(ctrl: int, src: list) -> list:
    """Lane i of the result holds src[k] for the source lane k that DPP
    control `ctrl` names (bound_ctrl on: an out-of-row source reads 0)."""
    out = []
    for i in range(WAVE):
        row, r = divmod(i, 16)
        if ctrl <= 0xFF:  # quad_perm: lane i takes lane 4*(i//4) + sel[i%4]
            k = (i & ~3) | ((ctrl >> (2 * (i & 3))) & 3)
        elif 0x111 <= ctrl <= 0x11F:  # row_shr:n
            n = ctrl - 0x110
            k = i - n if r >= n else None
        elif ctrl == 0x140:  # row_mirror
            k = row * 16 + 15 - r
        elif ctrl == 0x141:  # row_half_mirror
            k = row * 16 + (r & 8) + 7 - (r & 7)
        else:
            raise ValueError(hex(ctrl))
        out.append(0 if k is None else src[k])
    return out


LANES = list(range(WAVE))


@pytest.mark.parametrize("m,ctrls", [(1, [0xB1]), (2, [0x4E]), (4, [0x1B, 0x141]), (8, [0x141, 0x140])])
def test_xor_moves(m, ctrls):
    v = LANES
    for c in ctrls:
        v = dpp(c, v)
    assert v == [i ^ m for i in LANES]


@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_shift_up_within_rows(n):
    v = dpp(0x110 + n, LANES)
    for i in LANES:
        if i % 16 >= n:
            assert v[i] == i - n
        else:
            assert v[i] == 0


def test_previous_lane_in_groups_of_four_and_eight():
    v = dpp(0x111, LANES)
    for g in (4, 8):
        for i in LANES:
            if i % g:  # what lane 0 of a group receives is not used
                assert v[i] == i - 1


def test_last_lane_broadcast():
    # groups of 4: quad_perm [3,3,3,3]
    assert dpp(0xFF, LANES) == [(i | 3) for i in LANES]
    # groups of 8: each quad's last lane, then the other quad's by the half
    # mirror, taken by the lower quad
    a = dpp(0xFF, LANES)
    b = dpp(0x141, a)
    got = [b[i] if i % 8 < 4 else a[i] for i in LANES]
    assert got == [(i | 7) for i in LANES]


def test_sources_use_these_controls():
    # the kernels' DPP controls are the ones modelled above
    used = set()
    for f in ("knn.hip", "clip.hip"):
        used |= {int(x, 16) for x in re.findall(r"dpp_mov<(0x[0-9A-Fa-f]+)>", (CSRC / f).read_text())}
    assert used <= {0xB1, 0x4E, 0x1B, 0xFF, 0x111, 0x112, 0x114, 0x118, 0x140, 0x141}
    assert {0xB1, 0x4E, 0x1B, 0x141, 0x140, 0x111, 0xFF} <= used
