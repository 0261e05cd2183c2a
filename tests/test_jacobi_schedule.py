"""Host-side checks of the blocked cyclic Jacobi order that the split
eigensolver kernels (k_jacobi_rot, k_apply_rot) rely on, simulated in Python
for every padded size they accept (m = 4 .. 256):

* every pair of indices is rotated exactly once per sweep;
* the quartet tiles of round r + 1 lie in the off-diagonal blocks that the
  rotation kernel's first wave takes in round r (quartet pairs (q - 1, q + 1),
  (0, 1), (nq - 2, nq - 1)), so that wave may solve round r + 1 before the
  other waves finish round r;
* the apply kernel's lane moves (X block to lane q - 1, Y block to lane q + 1,
  lane 0 keeping block 0 and taking lane 1's X as its Y, the last quartet's Y
  becoming its X) reproduce each round's quartets and return to the starting
  arrangement after a sweep.
"""

import pytest


def rr(pos, step, M):
    """Block at position pos in round step (position 0 fixed, 1 .. M-1 advance)."""
    if pos == 0:
        return 0
    return 1 + (pos - 1 + step) % (M - 1)


def quartets(m, rd):
    nb2, nq = m // 2, m // 4
    return [(rr(q, rd, nb2), rr(nb2 - 1 - q, rd, nb2)) for q in range(nq)]


SIZES = list(range(4, 260, 4))


@pytest.mark.parametrize("m", SIZES)
def test_every_pair_once_per_sweep(m):
    nb2 = m // 2
    seen = {}
    for k in range(nb2):  # block step
        seen[(2 * k, 2 * k + 1)] = seen.get((2 * k, 2 * k + 1), 0) + 1
    for rd in range(nb2 - 1):
        blocks = [b for qb in quartets(m, rd) for b in qb]
        assert sorted(blocks) == list(range(nb2)), "a round's quartets partition the blocks"
        for X, Y in quartets(m, rd):
            for i in (2 * X, 2 * X + 1):
                for j in (2 * Y, 2 * Y + 1):
                    key = (min(i, j), max(i, j))
                    seen[key] = seen.get(key, 0) + 1
    assert len(seen) == m * (m - 1) // 2
    assert set(seen.values()) == {1}


def critical_pairs(nq):
    ncrit = nq if nq >= 3 else (1 if nq == 2 else 0)
    out = set()
    for lane in range(ncrit):
        a = 0 if lane == 0 else (nq - 2 if lane == nq - 1 else lane - 1)
        b = 1 if lane == 0 else (nq - 1 if lane == nq - 1 else lane + 1)
        out.add((a, b))
    return out


@pytest.mark.parametrize("m", SIZES)
def test_next_round_tiles_in_first_wave_blocks(m):
    nq = m // 4
    crit = critical_pairs(nq)
    pred = {(a, b) for a in range(nq) for b in range(a + 1, nq)
            if b == a + 2 or (a == 0 and b == 1) or (a == nq - 2 and b == nq - 1)}
    assert crit == pred
    for rd in range(m // 2 - 2):
        where = {}
        for q, (X, Y) in enumerate(quartets(m, rd)):
            where[X] = q
            where[Y] = q
        for X, Y in quartets(m, rd + 1):
            a, b = sorted((where[X], where[Y]))
            assert a != b and (a, b) in crit


@pytest.mark.parametrize("m", SIZES)
def test_apply_lane_moves_follow_the_rounds(m):
    nb2, nq = m // 2, m // 4
    lanes = [(q, nb2 - 1 - q) for q in range(nq)]  # starting arrangement (round 0)
    for rd in range(nb2 - 1):
        assert lanes == quartets(m, rd)
        if nq > 1:
            X = [x for x, _ in lanes]
            Y = [y for _, y in lanes]
            nxt = []
            for q in range(nq):
                from_next = X[q + 1] if q + 1 < nq else None
                from_prev = Y[q - 1] if q >= 1 else None
                if q == 0:
                    nxt.append((X[0], from_next))
                elif q == nq - 1:
                    nxt.append((Y[q], from_prev))
                else:
                    nxt.append((from_next, from_prev))
            lanes = nxt
    assert lanes == [(q, nb2 - 1 - q) for q in range(nq)]


def wave_step(X, Y, nq, half):
    """One round-to-round move of the apply kernel over a 64-lane wave: DPP
    wave_shl:1 (lane i reads i + 1) and wave_shr:1 (lane i reads i - 1), then
    the per-lane choices; half = 32 when two column sets share the wave."""
    L = len(X)
    shl = [X[i + 1] if i + 1 < L else 0 for i in range(L)]
    shr = [Y[i - 1] if i >= 1 else 0 for i in range(L)]
    nX, nY = list(X), list(Y)
    for lane in range(L):
        q = lane % half
        first, last = q == 0, q == nq - 1
        t = Y[lane] if last else shl[lane]
        nY[lane] = shl[lane] if first else shr[lane]
        nX[lane] = X[lane] if first else t
    return nX, nY


@pytest.mark.parametrize("m", SIZES)
def test_apply_wave_moves_with_two_column_sets(m):
    """The DPP moves over the whole wave keep each half's quartets right,
    also when two column sets share a wave (m <= 128): no active lane reads a
    value from the other half."""
    nb2, nq = m // 2, m // 4
    half = 32 if m <= 128 else 64
    sets = 64 // half
    # lanes past the last quartet carry a marker that must never reach an active lane
    X = [(lane // half, lane % half) if lane % half < nq else ("idle", lane) for lane in range(64)]
    Y = [(lane // half, nb2 - 1 - lane % half) if lane % half < nq else ("idle", lane) for lane in range(64)]
    for rd in range(nb2 - 1):
        for s in range(sets):
            got = [(X[s * half + q], Y[s * half + q]) for q in range(nq)]
            want = [((s, a), (s, b)) for a, b in quartets(m, rd)]
            assert got == want, (m, rd, s)
        if nq > 1:
            X, Y = wave_step(X, Y, nq, half)
    for s in range(sets):
        assert [(X[s * half + q], Y[s * half + q]) for q in range(nq)] == \
            [((s, q), (s, nb2 - 1 - q)) for q in range(nq)]
