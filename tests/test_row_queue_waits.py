"""Model check of the explicit memory waits of the fused row streams.

The edge and Gaussian5x5 streams read their input rows from a queue in LDS
filled by direct-to-LDS loads, and the corner stream does the same with a
one-dword queue.  The compiler does not order those loads against the LDS
reads, so each read is preceded by `s_waitcnt vmcnt(N)`: the wave may go on
while at most N vector-memory operations are outstanding, and since they
complete in issue order, the row is complete if at least N operations were
issued after its last load.  This test replays the order in which a stream
issues its loads and stores, for every band geometry that matters, and
checks that the immediate the device code picks never exceeds the number of
operations actually issued after the awaited load (it may be smaller: that
only waits longer).  The rules below restate the device code's formulas."""
import itertools

import pytest


def lds_rows_wait(NB, S, Q, y, y0, y1):
    """The immediate LdsRows::take waits with at output row y."""
    F = Q * S + (Q - 1) * NB
    A, B = Q * S, (Q - 1) * NB
    X, Y = max(A, B), min(A, B)
    n = min(y - y0, Q) * S + NB * (Q - 1 - min(max(y + Q - y1, 0), Q - 1))
    for imm in (F, X, Y):
        if n >= imm:
            return imm
    return 0


def replay_lds_rows(NB, S, Q, y0, y1):
    """Issue order of one band [y0, y1): returns, for each output row y, the
    number of operations issued after the last load of row y+2 at the moment
    of its wait, and the immediate used."""
    ops = []  # ("load", row) or ("store", row)
    issued_at = {}

    def issue(r):
        for _ in range(NB):
            ops.append(("load", r))
        issued_at[r] = len(ops)  # index just past the row's last load

    checks = []
    for k in range(Q):  # start(): rows y0-2 .. y0+Q-3, then wait for the first four
        issue(y0 - 2 + k)
    for r in range(y0 - 2, y0 + 2):  # vmcnt(NB*(Q-4)) before reading rows y0-2 .. y0+1
        checks.append((len(ops) - issued_at[r], NB * (Q - 4), "start", r))
    for k in range(4):  # refill()
        issue(y0 + Q - 2 + k)
    for y in range(y0, y1):
        younger = len(ops) - issued_at[y + 2]
        checks.append((younger, lds_rows_wait(NB, S, Q, y, y0, y1), "take", y))
        if y + Q + 2 <= y1 + 1:
            issue(y + Q + 2)
        for _ in range(S):
            ops.append(("store", y))
    return checks


@pytest.mark.parametrize("NB,S,Q", [(1, 1, 4), (1, 2, 4), (2, 1, 4), (1, 1, 8), (1, 2, 8), (2, 1, 8)])
def test_lds_rows_waits_never_exceed_the_issued_count(NB, S, Q):
    # every band height from 1 to 3Q+3, bands at the image top (y0 = 0) and
    # inside it; the image height only clamps row addresses, not the order
    for rows, y0 in itertools.product(range(1, 3 * Q + 4), (0, 1, 5, 40)):
        for younger, imm, where, y in replay_lds_rows(NB, S, Q, y0, y0 + rows):
            assert imm <= younger, (NB, S, Q, rows, y0, where, y, imm, younger)


def test_lds_rows_steady_state_uses_the_full_count():
    # in the middle of a long band the wait lets every later operation stay
    # outstanding (no needless waiting)
    for NB, S, Q in [(1, 1, 4), (1, 2, 4), (2, 1, 4)]:
        checks = replay_lds_rows(NB, S, Q, 0, 64)
        mid = [(younger, imm) for younger, imm, where, y in checks if where == "take" and 10 <= y < 50]
        assert all(imm == younger == Q * S + (Q - 1) * NB for younger, imm in mid), (NB, S, Q, mid[:3])


def corner_wait(stores):
    """The immediate RowQueue::take (corner stream, eight rows) waits with."""
    if stores >= 8:
        return 15
    if stores >= 4:
        return 11
    return 7


def replay_corner(y0, y1, H, kQ=8):
    """Issue order of one corner band: input rows enter the queue kQ ahead;
    the band starts with takes that fill the five-row ring (no stores between
    them), then alternates one output store and one take, and stops taking
    once the rows pass the image."""
    ops, issued_at, checks = [], {}, []
    stores = 0

    def issue(r):
        ops.append(("load", r))
        issued_at[r] = len(ops)

    def take(r):
        checks.append((len(ops) - issued_at[r], corner_wait(stores), r))
        issue(r + kQ)

    nr = max(y0 - 2, 0)
    for k in range(kQ):
        issue(nr - 1 + k)
    take(nr - 1)
    take(nr)
    take(nr + 1)

    def next_h(r):  # a horizontal-sum row r < H takes input row r + 2
        if r < H:
            take(r + 2)

    if y0 - 2 < 0:
        next_h(0)
        for j in range(5):
            r = y0 - 2 + j
            if r > 0:
                next_h(r)
    else:
        for j in range(5):
            next_h(y0 - 2 + j)
    for y in range(y0, y1):
        ops.append(("store", y))
        stores += 1
        next_h(y + 3)
    return checks


def test_corner_waits_never_exceed_the_issued_count():
    for H in (1, 2, 3, 5, 9, 30):
        for rows in range(1, 14):
            for y0 in range(0, H, rows):
                y1 = min(y0 + rows, H)
                for younger, imm, r in replay_corner(y0, y1, H):
                    assert imm <= younger, (H, rows, y0, r, imm, younger)
