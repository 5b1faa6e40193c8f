"""MI355X (gfx950) solver for the metric-constrained correlation-clustering LP.

Submodules: ``instances`` (seeded synthetic inputs), ``ccproj`` (binding of
the HIP library), ``build`` (in-tree hipcc build).  Nothing is imported here
so that the input generators load without the GPU library."""
