"""Measurement infrastructure (not part of the simulation path): a CPU replay of the
BVH walk over the GPU-built tree, used for the algorithmic bytes of the roofline."""
