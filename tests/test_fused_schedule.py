"""CPU model of the dispatch schedule of the fused forward pass (no GPU).

A fused pass launches gx*gy chunk-elimination units (strip group by strip
group, each XCD taking a contiguous range of groups), followed -- in the
one-launch form -- by the ex*gy re-solve units.  The last `nlast` elimination
units of a group to finish wait until the whole group has finished, then
solve its separator systems; a re-solve unit waits for the separator systems
of the one or two groups its 64 strips belong to.  The model dispatches the
units the way the hardware does (linear workgroup id i goes to XCD i mod 8,
each XCD starts its workgroups in order, a bounded number resident at once),
runs them with random durations and checks that every unit finishes whenever
the host's admission rule (2 * nlast <= resident workgroups per XCD) holds,
under two dispatcher models: one global in-order dispatcher that stalls while
the target XCD is full, and eight independent per-XCD dispatchers.  It also
checks that the model does find the deadlock the rule exists to prevent.
"""
import math
import random

import pytest

XCDS = 8


def xcd_rank(lin, n):
    """Logical position of dispatch slot `lin` of `n` (the device remap)."""
    x, idx = lin % XCDS, lin // XCDS
    q, rem = divmod(n, XCDS)
    return x * q + min(x, rem) + idx


def build_units(W, r, gy, Q, full):
    nK = W - 2 * r                          # stride-1 strips
    OW = 64 - 2 * r                         # columns owned by a re-solve unit
    gx = math.ceil(nK / 64)
    ex = math.ceil(W / OW)
    nlast = min(gy, math.ceil(64 / Q))
    nred = gx * gy
    units = []
    for lin in range(nred):
        units.append(("R", xcd_rank(lin, nred) // gy))
    if full:
        for e in range(ex * gy):
            bx = xcd_rank(e, ex * gy) // gy
            ki_lo = min(max(0, bx * OW - 2 * r), nK - 1)
            ki_hi = min(ki_lo + 63, nK - 1)
            units.append(("E", (ki_lo // 64, ki_hi // 64)))
    return units, gx, nlast


def simulate(units, gx, gy, nlast, slots, model, seed, max_steps=200000):
    """True when every unit finishes, False on a deadlock."""
    rng = random.Random(seed)
    red = [0] * gx
    ifc = [0] * gx
    n = len(units)
    queues = [[i for i in range(n) if i % XCDS == x] for x in range(XCDS)]
    heads = [0] * XCDS
    nxt = 0                                  # global dispatcher position
    resident = [[] for _ in range(XCDS)]     # [unit, state, remaining]
    done = 0
    idle = 0
    for _ in range(max_steps):
        progressed = False
        # dispatch
        if model == "global":
            while nxt < n and len(resident[nxt % XCDS]) < slots:
                resident[nxt % XCDS].append([nxt, "run", rng.randint(1, 4)])
                nxt += 1
                progressed = True
        else:
            for x in range(XCDS):
                while heads[x] < len(queues[x]) and len(resident[x]) < slots:
                    resident[x].append([queues[x][heads[x]], "run", rng.randint(1, 4)])
                    heads[x] += 1
                    progressed = True
        # one step of every resident unit
        for x in range(XCDS):
            keep = []
            for u in resident[x]:
                kind, arg = units[u[0]]
                st = u[1]
                if st == "run":
                    u[2] -= 1
                    progressed = True
                    if u[2] == 0:
                        if kind == "R":
                            ticket = red[arg]
                            red[arg] += 1
                            if ticket < gy - nlast:
                                done += 1
                                continue
                            u[1] = "wait"
                        else:
                            done += 1
                            continue
                elif st == "wait":
                    if kind == "R" and red[arg] == gy:
                        u[1], u[2] = "iface", rng.randint(1, 3)
                        progressed = True
                    elif kind == "E" and ifc[arg[0]] >= nlast and ifc[arg[1]] >= nlast:
                        u[1], u[2] = "run2", rng.randint(1, 4)
                        progressed = True
                elif st in ("iface", "run2"):
                    u[2] -= 1
                    progressed = True
                    if u[2] == 0:
                        if st == "iface":
                            ifc[arg] += 1
                        done += 1
                        continue
                keep.append(u)
            resident[x] = keep
        if done == n:
            return True
        idle = 0 if progressed else idle + 1
        if idle > 2:
            return False
    raise AssertionError("simulation did not settle")


SHAPES = [
    # (W, r, rows L, R, Q): the 1080p frames at the tuned chunk shapes, a
    # narrow frame (one strip group), a tall frame (many chunks per strip).
    (1920, 1, 1080, 10, 4), (1080, 1, 1920, 10, 4), (1920, 1, 1080, 4, 8),
    (1080, 1, 1920, 8, 8), (130, 1, 900, 6, 4), (700, 2, 3000, 4, 4), (4000, 1, 64, 8, 2),
]


@pytest.mark.parametrize("model", ["global", "per_xcd"])
@pytest.mark.parametrize("full", [True, False])
@pytest.mark.parametrize("shape", SHAPES)
def test_admitted_launches_finish(shape, full, model):
    W, r, L, R, Q = shape
    gy = math.ceil(math.ceil(L / R) / Q)
    units, gx, nlast = build_units(W, r, gy, Q, full)
    for slots in (2 * nlast, 2 * nlast + 7, 64, 128):   # resident workgroups per XCD
        for seed in range(3):
            assert simulate(units, gx, gy, nlast, slots, model, seed), (shape, slots, seed)


@pytest.mark.parametrize("model", ["global", "per_xcd"])
def test_model_finds_the_deadlock_the_rule_prevents(model):
    # Fewer resident slots than waiting last finishers: a group's remaining
    # units can never start while its waiters hold every slot of the XCD.
    W, r, L, R, Q = 1920, 1, 1080, 10, 4
    gy = math.ceil(math.ceil(L / R) / Q)
    units, gx, nlast = build_units(W, r, gy, Q, True)
    assert not simulate(units, gx, gy, nlast, nlast // 2, model, 0)
