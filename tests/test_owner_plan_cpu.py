"""Host-side check of the owner-computes tiles' order of additions (no GPU).

A tile owns a 16 x 8 x 4 box of nodes (the last tile in a direction also the
mesh's last node plane in it) and computes the 17 x 9 x 5 elements touching the
box.  Wave w computes element layer w + 1 and the w-th quarter of layer 0, in
three steps of 64 lanes; pass L adds lower corners of the main layer, pass U1
upper corners of the main layer and of the quarters of waves 0 and 2, pass U2
the quarters of waves 1 and 3.  The sum at a node is bitwise reproducible when,
in every pass, the node receives additions from one wavefront only, and within
one instruction (one step, one corner) the lanes' nodes are distinct.  This
test walks that assignment for interior and edge tiles and checks those
properties, and that every owned node receives each of its element
contributions exactly once (8 for a node inside the mesh).
"""
import collections
import itertools

import pytest

OX, OY, OZ = 16, 8, 4
EX, EY = OX + 1, OY + 1
NL = EX * EY            # elements per layer of the box
NQ = NL // 4            # layer-0 quarter


def lanes(w):
    """(step, lane) -> element (ea, eb, ec) of wave w, or None for an empty lane."""
    out = {}
    for k, lane in itertools.product(range(3), range(64)):
        j = 64 * k + lane
        if j < NL:
            out[(k, lane)] = (j % EX, j // EX, w + 1, True)
        else:
            q = NQ * w + j - NL
            q1 = NL if w == 3 else NQ * (w + 1)
            out[(k, lane)] = (q % EX, q // EX, 0, False) if q < q1 else None
    return out


def walk(last_x, last_y, last_z, first_x=False, first_y=False, first_z=False):
    """Additions per (pass, node): the wavefronts that add, and per node the
    multiset of (element, corner) contributions."""
    hx, hy, hz = OX + last_x, OY + last_y, OZ + last_z
    writers = collections.defaultdict(set)      # (pass, node) -> waves
    per_instr = collections.defaultdict(list)   # (pass, wave, step, corner) -> nodes
    contrib = collections.defaultdict(list)     # node -> [(element, corner)]
    for w in range(4):
        for (k, lane), el in lanes(w).items():
            if el is None:
                continue
            ea, eb, ec, main = el
            # elements outside the mesh (the box's shell beyond the first planes)
            if (first_x and ea == 0) or (first_y and eb == 0) or (first_z and ec == 0):
                continue
            for a in range(8):
                na, nb, nc = ea + (a & 1), eb + ((a >> 1) & 1), ec + (a >> 2)
                if not (1 <= na <= hx and 1 <= nb <= hy and 1 <= nc <= hz):
                    continue
                if a < 4:
                    p = "L"
                else:
                    p = "U1" if (main or w % 2 == 0) else "U2"
                node = (na, nb, nc)
                writers[(p, node)].add(w)
                per_instr[(p, w, k, a)].append(node)
                contrib[node].append(((ea, eb, ec), a))
    return writers, per_instr, contrib, (hx, hy, hz)


@pytest.mark.parametrize("last", [(0, 0, 0), (1, 0, 0), (0, 1, 1), (1, 1, 1)])
@pytest.mark.parametrize("first", [(False, False, False), (True, True, True)])
def test_owner_order_single_writer(last, first):
    writers, per_instr, contrib, (hx, hy, hz) = walk(*last, *first)
    # one wavefront per node and pass
    assert all(len(ws) == 1 for ws in writers.values())
    # distinct nodes within an instruction
    assert all(len(ns) == len(set(ns)) for ns in per_instr.values())
    # every owned node gets each contribution once: the elements around it that
    # lie inside the mesh (8, or fewer on the mesh's first planes)
    for na, nb, nc in itertools.product(range(1, hx + 1), range(1, hy + 1), range(1, hz + 1)):
        cs = contrib[(na, nb, nc)]
        assert len(cs) == len(set(cs))
        want = 0
        for da, db, dc in itertools.product((0, 1), repeat=3):
            ea, eb, ec = na - da, nb - db, nc - dc
            inside = (ea >= 0 and eb >= 0 and ec >= 0 and ea < OX + 1 and eb < OY + 1
                      and ec < OZ + 1)
            if first[0] and ea == 0 or first[1] and eb == 0 or first[2] and ec == 0:
                inside = False
            # beyond the mesh's last plane there are no elements
            if last[0] and ea == OX + 1 or last[1] and eb == OY + 1 or last[2] and ec == OZ + 1:
                inside = False
            want += inside
        assert len(cs) == want, ((na, nb, nc), len(cs), want)


def test_owner_quarters_share_no_node():
    """Quarters 0 and 2, and 1 and 3, of layer 0 touch disjoint node sets (the
    reason the two passes U1 and U2 suffice for layer 0)."""
    def nodes(w):
        q1 = NL if w == 3 else NQ * (w + 1)
        out = set()
        for q in range(NQ * w, q1):
            ea, eb = q % EX, q // EX
            out |= {(ea + i, eb + j) for i in (0, 1) for j in (0, 1)}
        return out
    assert not nodes(0) & nodes(2)
    assert not nodes(1) & nodes(3)
    assert nodes(0) & nodes(1)  # adjacent quarters do share nodes
