"""CPU model of the sliding-column register scheme of the separable and
symmetric blur kernels (circular buffer of 2R+1 pending outputs).  Checks,
for every radius the library instantiates, that each emitted output receives
exactly the contributions a = R..-R in that order starting with an
assignment, that no slot is reused while its output is pending, and that
every LDS row read lies inside the padded tile."""
import pytest

TH = 32


def _model(R):
    NW = 2 * R + 1
    LH = TH + 2 * R
    NG = (LH + NW - 1) // NW
    LH_PAD = NG * NW
    slot_owner = [None] * NW
    contrib = {}
    emitted = []
    for gi in range(NG):
        for k in range(NW):
            t = gi * NW + k
            assert 0 <= t < LH_PAD
            # the 2R+1 outputs fed by one row occupy distinct slots
            assert len({((k - R + a) % NW + NW) % NW for a in range(-R, R + 1)}) == NW
            for a in range(R, -R - 1, -1):
                v = t - R + a
                s = ((k - R + a) % NW + NW) % NW
                assert s == v % NW
                if a == R:
                    # assignment starts output v; the slot's previous output is done
                    prev = slot_owner[s]
                    assert prev is None or prev + 2 * R < t
                    slot_owner[s] = v
                    contrib[v] = [a]
                else:
                    # outputs above the tile (v < 0) start mid-window: junk, never emitted
                    if v >= 0:
                        assert slot_owner[s] == v
                        contrib[v].append(a)
            vd = t - 2 * R
            if 0 <= vd < TH:
                s = ((k - R - R) % NW + NW) % NW
                assert slot_owner[s] == vd
                assert contrib[vd] == list(range(R, -R - 1, -1))
                emitted.append(vd)
    return emitted


@pytest.mark.parametrize("R", list(range(0, 13)))
def test_sliding_scheme(R):
    assert _model(R) == list(range(TH))
