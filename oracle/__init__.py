"""CPU oracle for incremental octree LOD insertion (SimLOD, arXiv 2310.03567).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package: only ``tests/``, the smoke check
in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` use it.  It
shares no code with the HIP library and imports nothing from it.

Two independent implementations of the same result live here:

* ``definition.build`` (O1) -- the octree written out as its plain recursive
  definition over the cumulative point sequence (numpy, vectorised per node).
* ``incremental`` (O2) -- the classic sequential top-down inserter that
  splits a leaf as soon as it overflows and re-inserts its points from the
  split node downward (plain C, one thread), as described for CPU-based
  approaches in the paper's section "Expanding the Octree".

Both emit the canonical form defined in ``canonical``.  The paper's batch
passes (count/split, sample, allocate, store) reach exactly this result
because (i) a leaf's counter covers its stored points plus the new ones, so
"inner" is equivalent to "the node's region holds more than T points", and
(ii) every point held by a node that turns inner is re-sampled through it via
the spill buffer, so with the minimum-key voxel representative the result
depends only on the cumulative sequence, not on how it was cut into batches.

Pins (see ``tests/test_oracle_*.py``): O1 against O2 exhaustively on tiny
inputs, closed forms, a hand-worked example in ``tests/golden``, invariants
checked by an independent brute-force checker, batch-partition invariance,
and the backlog bound from section "Voxel Sampling".
"""

from .canonical import (  # noqa: F401
    LodConfig,
    CanonicalTree,
    NODE_DTYPE,
    POINT_DTYPE,
    assert_trees_equal,
    path_depth,
    subtree,
    trees_equal,
)
