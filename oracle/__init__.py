"""FP64 CPU oracle for the block-iterative CT solver (CSGD / GCSGD).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package: only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark use it.  It shares no code
with the HIP library; the only common dependency is the seeded input module
(geometry vectors, partitions, phantoms), which contains none of the method's
arithmetic.

Contents
--------
rays      -- one FP64 line per detector bin from the per-view vectors.
siddon    -- explicit system matrix A (Sec. II-A: A_ij = intersection length
             of ray i with voxel j) by a Siddon traversal (C, FP64), plus the
             closed-form single-pair clip length used to pin it.
sampler   -- the data-independent block schedule of Alg. 5 / Alg. 6
             (column order, weighted row-block draws without replacement,
             groups, relaxation beta) driven by a counter-based SplitMix64.
csgd      -- Alg. 4 / 5 / 6 step by step on explicit sparse sub-blocks.

Functions whose result has no independent pin say "parity unpinned" in
their docstring.
"""
