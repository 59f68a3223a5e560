"""CPU pins for the oracle's brute-force fewest-strips count (Sec. 3.1, the
optimal GTS): closed forms that exercise each constraint -- a path needs no
restart, a triangle with three neighbours forks, a closed surface or ring has
a cycle to break, disjoint triangles need one strip each."""
import numpy as np

import meshgen
import oracle as O


def test_paths_and_disjoint():
    for k in (1, 2, 5, 16):
        assert O.min_strips(meshgen.fan(k).tri) == 1
    for k in (1, 3, 16):
        assert O.min_strips(meshgen.disjoint(k).tri) == k


def test_fork_star():
    """A centre triangle with a neighbour on each edge: one of the three
    neighbours must start a strip of its own -> 2 strips."""
    tri = np.array([(0, 1, 2), (1, 0, 3), (2, 1, 4), (0, 2, 5)], np.uint32)
    assert O.min_strips(tri) == 2
    # double star: two forks joined -> 6 triangles, 2 strips (a path of 4 + 2 spares joined pairwise)
    tri2 = np.array([(0, 1, 2), (1, 0, 3), (2, 1, 4), (0, 2, 5), (3, 0, 6), (1, 3, 7)], np.uint32)
    assert O.min_strips(tri2) == 2


def test_cycles():
    """A closed ring of k triangles around a hub and the tetrahedron surface:
    every triangle has two (ring) or three (tetrahedron) neighbours in a
    cycle; one path covers all -> 1 strip."""
    for k in (3, 6, 9):
        tri = np.array([(0, 1 + i, 1 + (i + 1) % k) for i in range(k)], np.uint32)
        assert O.min_strips(tri) == 1
    tet = np.array([(0, 1, 2), (0, 3, 1), (1, 3, 2), (0, 2, 3)], np.uint32)
    assert O.min_strips(tet) == 1


def test_two_pieces_of_a_grid():
    """4x2 grid of quads (16 triangles): a snake visits all -> 1 strip.  With
    one quad's two triangles flipped to the other winding, the edges between
    that quad and the rest are no longer crossable: the quad is a piece of its
    own (one strip) and the count is the rest's count plus one."""
    m = meshgen.grid(4, 2, meshgen.rng_for(9, 1), permute=False)
    assert m.ntri == 16
    assert O.min_strips(m.tri) == 1
    bad = m.tri.copy()
    bad[0] = bad[0][[0, 2, 1]]
    bad[1] = bad[1][[0, 2, 1]]
    assert O.min_strips(bad[:2]) == 1
    assert O.min_strips(bad) == O.min_strips(bad[2:]) + 1
