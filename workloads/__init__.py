"""Seeded synthetic workloads: meshes, trace maps and primitive flow fields.

This package is shared by the CPU oracle and the GPU path as a source of
*inputs only*.  It holds none of the method's arithmetic: no entropy-variable
map, no flux, no quadrature, no basis.  It produces

* meshes as per-element vertex coordinates plus integer lattice data
  (``meshes``),
* integer trace maps for the HDG / EDG / IEDG trace spaces, which differ only
  in which trace nodes are shared (``meshes.trace_map``),
* primitive fields (density, velocity, pressure) and their spatial gradients
  at caller-given points, with seeded smooth and per-node noise (``fields``),
* the named workload recipes (``configs``).

Converting primitives to entropy variables (and gradients to q) is part of
the method and happens on each side separately.
"""
