"""Host model of the full-row strip solve's schedule (kernels_solve.hip:
strip_solve_pf_kernel and its launch table), checked on the CPU.

The kernel solves every strip by the twisted block substitution: forward
products from both ends towards the middle line, the middle product, then
backward products outwards, one product from above and one from below per
step, the team of workgroups of a strip separated by a counter barrier
after every step.  Member w of a team owns rows [r0, r1) of every product;
a step's rows of both products form one list dealt round-robin to the
waves, PR rows per wave held in registers, the rest streamed.  Every tile
stages the forward results of the next step's backward rows in LDS while
the barrier is pending; a backward row then takes its forward result from
there.

The model replays every member's steps with the kernel's index arithmetic
and checks, for every tile shape of the launch table, several line widths,
strip widths and team sizes:
  * every row of every product is computed exactly once, by its owner;
  * every vector element a step reads from x was written at an earlier
    step (so behind at least one team barrier), with the value the
    substitution needs there (forward result, or final result for the
    backward sweep);
  * a staged forward result was written by the same member at an earlier
    step, is still the forward result when staged, and is read back by the
    same member at the next step from the slot it was staged into;
  * staging indices stay in the LDS area the launch allocates.
"""
import numpy as np
import pytest

TOP_F, BOT_F, MID, TOP_B, BOT_B = range(5)


def tw_steps(nx):
    return 2 * (nx - 1 - (nx - 1) // 2) + 1


def tw_step(nx, s):
    m = (nx - 1) // 2
    nb = nx - 1 - m
    if s < nb:
        return (s if s < m else -1, TOP_F, nx - 1 - s, BOT_F)
    if s == nb:
        return (m, MID, -1, BOT_F)
    e = s - nb - 1
    return (m - 1 - e if m - 1 - e >= 0 else -1, TOP_B, m + 1 + e, BOT_B)


def backward(kind):
    return kind in (TOP_B, BOT_B)


# (fp32, NW, NCH, PR) of every full-row tile shape in the launch table
SHAPES = [
    (1, 8, 3, 8), (1, 8, 3, 3), (1, 16, 3, 2),
    (1, 8, 9, 5), (1, 8, 9, 2), (1, 16, 9, 2), (1, 8, 9, 9),
    (1, 8, 17, 3), (1, 8, 17, 1), (1, 16, 17, 1), (1, 8, 17, 4),
    (1, 8, 33, 1),
    (0, 8, 3, 4), (0, 16, 3, 4),
    (0, 8, 9, 3), (0, 8, 9, 1), (0, 16, 9, 1), (0, 8, 9, 4),
    (0, 8, 17, 1),
]


def lds_bytes(n, fp32, staged):
    e2 = 8 if fp32 else 16
    return 2 * n * e2 + (2 * n * 16 if staged else 0)


def simulate(n, nx, team, NW, PR, staged):
    """Replays one strip; returns the number of checks made."""
    S = tw_steps(nx)
    # x state per line: -1 unwritten, 1 forward result, 2 final result;
    # stamp = step of the last write, owner = member that wrote each row
    state = np.full((nx, n), -1, int)
    stamp = np.full((nx, n), -1, int)
    owner = np.full((nx, n), -1, int)
    rpw = -(-n // team)
    checks = 0
    staged_slots = [None] * team   # member -> {(p, q): (line, row)}
    for st in range(S):
        lt, kt, lb, kb = tw_step(nx, st)
        prods = [(p, L, k) for p, (L, k) in enumerate(((lt, kt), (lb, kb))) if L >= 0]
        # vector phase (every member reads whole neighbour lines)
        for p, L, k in prods:
            for nb_line, needed in (((L - 1), 1 if k in (TOP_F, MID) else 2),
                                    ((L + 1), 1 if k in (BOT_F, MID) else 2)):
                uses = ((k in (TOP_F, MID, BOT_B) and nb_line == L - 1 and L > 0) or
                        (k in (BOT_F, MID, TOP_B) and nb_line == L + 1 and L < nx - 1))
                if not uses:
                    continue
                assert np.all(stamp[nb_line] < st), (st, L, k)
                assert np.all(state[nb_line] == needed), (st, L, k, nb_line)
                checks += 1
        writes = []
        for w in range(team):
            r0 = min(n, w * rpw)
            r1 = min(n, r0 + rpw)
            R = r1 - r0
            ents = [(0, r0 + i) for i in range(R)] if lt >= 0 else []
            ents += [(1, r0 + i) for i in range(R)] if lb >= 0 else []
            taken = np.zeros(len(ents), int)
            for wave in range(NW):
                rhos = [wave + NW * u for u in range(PR)]
                rho = wave + NW * PR
                while rho < len(ents):
                    rhos.append(rho)
                    rho += NW
                for rho in rhos:
                    if rho >= len(ents):
                        continue
                    taken[rho] += 1
                    p, r = ents[rho]
                    L, k = (lt, kt) if p == 0 else (lb, kb)
                    if backward(k):
                        assert state[L, r] == 1 and owner[L, r] == w
                        if staged:
                            # finish_row's slot: product 0 iff L is the line from above
                            ps = 0 if (lt >= 0 and L == lt) else 1
                            q = r - r0
                            assert 0 <= ps * n + q < 2 * n
                            assert staged_slots[w][(ps, q)] == (L, r)
                        writes.append((L, r, 2, w))
                    else:   # the middle product is final at once
                        writes.append((L, r, 2 if k == MID else 1, w))
                    checks += 1
            assert np.all(taken == 1)
        for L, r, v, w in writes:
            state[L, r] = v
            stamp[L, r] = st
            owner[L, r] = w
        if st == S - 1:
            break
        # publish: stage the next step's forward results of backward rows
        nlt, nkt, nlb, nkb = tw_step(nx, st + 1)
        for w in range(team):
            r0 = min(n, w * rpw)
            R = min(n, r0 + rpw) - r0
            slots = {}
            if staged:
                for p, (L, k) in enumerate(((nlt, nkt), (nlb, nkb))):
                    if L < 0 or not backward(k):
                        continue
                    for q in range(R):
                        assert p * n + q < 2 * n
                        assert state[L, r0 + q] == 1 and owner[L, r0 + q] == w
                        assert stamp[L, r0 + q] <= st
                        slots[(p, q)] = (L, r0 + q)
            staged_slots[w] = slots
    assert np.all(state == 2) or nx == 1
    return checks


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "f%d_%dw_%dch_pr%d" % s)
def test_full_row_schedule_is_race_free_and_in_bounds(shape):
    fp32, NW, NCH, PR = shape
    # line lengths: the shape's largest and a ragged one
    for n in sorted({64 * NCH, 64 * (NCH - 1) + 17}):
        # the staging area sits behind the two vectors in dynamic LDS
        assert lds_bytes(n, fp32, True) <= 160 * 1024
        for nx in (3, 4, 6, 33, 34):
            for team in (1, 3, 4, 16):
                assert simulate(n, nx, team, NW, PR, True) > 0
