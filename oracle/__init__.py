"""CPU oracle for the Octree-GS render path.  Test infrastructure: imported
only by tests, the smoke check and the benchmark's CPU-baseline leg."""
