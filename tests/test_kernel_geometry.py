"""CPU model of the streaming sliding-column scheme of the separable,
symmetric and uniform-disk blur kernels (circular buffer of 2R+1 pending
outputs, a register ring of prefetched rows, a centre ring, a two-row LDS
buffer).  Checks, for every radius the library instantiates, that the strip
height fills whole row groups, that each emitted output receives exactly the
contributions a = R..-R in that order starting with an assignment, that no
output or prefetch slot is reused while still pending, that every interior
row is handled once, and that every LDS access lies inside the row buffer.
Strips may also walk bottom-up: the row mapping then still visits every
interior row once and completes every output row from the 2R + 1 input rows
centred on it.  A strip whose rows all lie inside the image runs the row
groups between its first and its last without the per-row tests: every one
of those tests holds there, for every radius, strip height and direction."""
import pytest

KTH, KTW, PREFETCH = 32, 64, 2


def strip_group(R):
    """Mirror of strip_group(): a multiple of 2R + 1 of at least 4 rows."""
    NW = 2 * R + 1
    return NW * ((4 + 2 * R) // NW)


def strip_th(R, tall=False, short=False):
    """Mirror of strip_th(): smallest height >= 32 (tall strips: >= 64, short
    strips: >= 8) with (height + 2R) a multiple of the group size."""
    GS = strip_group(R)
    base = 2 * KTH if tall else (KTH // 4 if short else KTH)
    return GS * ((base + 2 * R + GS - 1) // GS) - 2 * R


def _model(R, tall=False):
    NW = 2 * R + 1
    TH = strip_th(R, tall)
    LH = TH + 2 * R
    LW = KTW + 2 * R
    GS = strip_group(R)
    base = 2 * KTH if tall else KTH
    assert GS % NW == 0 and GS >= 4
    assert TH >= base and TH < base + GS and LH % GS == 0
    NG = LH // GS
    D = min(GS, PREFETCH)
    slot_owner = [None] * NW
    contrib = {}
    emitted, interior = [], []
    ring = {}  # prefetch slot -> row it holds
    cen = {}   # centre slot -> input row
    for t in range(D):
        ring[t % GS] = t
    for gi in range(NG):
        for kg in range(GS):
            t = gi * GS + kg
            k = kg % NW
            assert k == t % NW
            # consume the prefetched row of this step, then refill D ahead
            assert ring.get(kg) == t, (t, ring)
            ring[(kg + D) % GS] = t + D
            if R <= t < R + TH:
                interior.append(t - R)
            # LDS: writes at lane and 64 + lane (lane < 2R), reads lane + 0..2R
            assert KTW - 1 < LW and (2 * R == 0 or KTW + 2 * R - 1 < LW)
            assert 63 + 2 * R < LW
            cen[k] = t
            for a in range(R, -R - 1, -1):
                v = t - R + a
                s = ((k - R + a) % NW + NW) % NW
                assert s == v % NW
                if a == R:
                    prev = slot_owner[s]
                    assert prev is None or prev + 2 * R < t
                    slot_owner[s] = v
                    contrib[v] = [a]
                else:
                    if v >= 0:
                        assert slot_owner[s] == v
                        contrib[v].append(a)
            if t >= 2 * R:
                vd = t - 2 * R
                s = ((k - R - R) % NW + NW) % NW
                assert slot_owner[s] == vd
                assert contrib[vd] == list(range(R, -R - 1, -1))
                # the centre of output row vd is input row vd + R
                assert cen[((k - R) % NW + NW) % NW] == vd + R
                emitted.append(vd)
    assert interior == list(range(TH))
    return emitted, TH


@pytest.mark.parametrize("tall", [False, True])
@pytest.mark.parametrize("R", list(range(0, 13)))
def test_streaming_scheme(R, tall):
    emitted, TH = _model(R, tall)
    assert emitted == list(range(TH))


@pytest.mark.parametrize("tall", [False, True])
@pytest.mark.parametrize("R", [0, 1, 3, 6, 12])
@pytest.mark.parametrize("up", [False, True])
def test_strip_row_mapping(R, up, tall):
    """Mirror of stream_strip's row_at / out_at for both walking directions."""
    TH = strip_th(R, tall)
    LH = TH + 2 * R
    y0 = 5 * TH
    ybase, ystep = (y0 + TH + R - 1, -1) if up else (y0 - R, 1)
    row_at = lambda t: ybase + ystep * t
    out_at = lambda t: ybase + ystep * (t - R)
    assert sorted(row_at(t) for t in range(LH)) == list(range(y0 - R, y0 + TH + R))
    assert sorted(row_at(t) for t in range(R, R + TH)) == list(range(y0, y0 + TH))
    assert sorted(out_at(t) for t in range(2 * R, LH)) == list(range(y0, y0 + TH))
    for t in range(2 * R, LH):
        # the window of steps t - 2R .. t holds the rows out_at(t) - R .. out_at(t) + R
        assert sorted(row_at(u) for u in range(t - 2 * R, t + 1)) == list(range(out_at(t) - R, out_at(t) + R + 1))


@pytest.mark.parametrize("mode", ["usual", "tall", "short"])
@pytest.mark.parametrize("R", list(range(0, 13)))
@pytest.mark.parametrize("up", [False, True])
def test_inner_groups_need_no_tests(R, mode, up):
    """Mirror of the tests stream_strip drops in the middle row groups of a
    strip inside the image: the prefetch of row t + D (in the image, inside
    the strip, interior-row load, output-row load) and the interior and
    output stores of step t all hold for every step of groups 1 .. NG - 2."""
    TH = strip_th(R, tall=mode == "tall", short=mode == "short")
    LH, GS = TH + 2 * R, strip_group(R)
    NG, D = LH // GS, min(GS, PREFETCH)
    # the conditions the kernel asserts at compile time
    assert GS > 2 * R and D + R <= GS
    h = 7 * TH + 3  # a ragged image height
    for y0 in range(0, h, TH):
        inside = y0 - R >= 0 and y0 + TH + R <= h
        ybase, ystep = (y0 + TH + R - 1, -1) if up else (y0 - R, 1)
        row_at = lambda t: ybase + ystep * t
        out_at = lambda t: ybase + ystep * (t - R)
        rows = [row_at(t) for t in range(LH)]
        assert inside == all(0 <= y < h for y in rows)
        if not inside:
            continue
        for gi in range(1, NG - 1):
            for kg in range(GS):
                t, tp = gi * GS + kg, gi * GS + kg + D
                row_ok = tp < LH and 0 <= row_at(tp) < h
                assert row_ok
                assert R <= tp < R + TH  # interior-row load of the prefetched row
                assert tp >= 2 * R and tp < LH and out_at(tp) < h  # output-row load
                assert R <= t < R + TH and row_at(t) < h  # interior store
                assert t >= 2 * R and out_at(t) < h  # output store
