"""FP64 CPU oracle for UniFrac distance matrices.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
anything here; only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may.  It shares no code with the GPU library: the only
common dependency is the seeded input generator module ``synth``.

Contents
--------
``unifrac``  plain definitions in numpy (FP64): postorder embedding, the two
             distance variants, PCoA row/grand means, the stripe layout.
``brute``    brute force for tiny trees: the tip set under every branch is found
             by walking parent pointers, with no postorder at all.
``core``     the same definitions in plain C (FP64, OpenMP over rows), used to
             time the CPU baseline and to check larger sample subsets.
``pcoa``     principal coordinates: the exact eigendecomposition of the
             double-centred matrix, and the randomized subspace iteration.
``placement`` the learned-placement encoder (projection, MLP, loss, Adam, kNN).
``mantel``   the Mantel test: Pearson / Spearman statistics and permutation
             p-values between two distance matrices.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
(hand-computed worked example, closed forms, brute force, scipy library
routines, invariants).  No function is "parity unpinned".
"""
from .unifrac import (  # noqa: F401
    TreeError, TableError, validate_tree, postorder, tips_of, embed_counts,
    embedding, dm, dm_pairs, pcoa_means, condensed_index, n_stripes,
    stripe_partner, to_stripes, gram_split_bf16,
)
from . import mantel, pcoa  # noqa: F401
