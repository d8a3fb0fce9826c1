"""FP64 CPU oracle for the global-placement hot path of arXiv 2403.09070 (test infrastructure).

This package is test infrastructure, not product code.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark import it; the HIP library never does, and it imports nothing
from the HIP path.  It shares with the GPU side only the seeded input generator.

Every function follows one passage of the paper and is written for a reader who checks it
against that passage: plain NumPy in float64, vectorised only where the vectorisation is an
obvious rewrite of a loop over instances, nets or bins.  Where the paper is silent or garbled,
the reading taken is stated in the function's docstring.

Modules
    geometry     bin grid, die depth, HBT weight alpha                       (Sec. V-A)
    attributes   partition, per-die sizes, macro size transition, pin offsets (Sec. III-A)
    density      exact-overlap density map; corner map + 3D prefix sum        (Sec. IV-A, Thm. 1)
    poisson      spectral Neumann Poisson solve: coefficients, phi, E, energy (Sec. III-A)
    density_grad field-gather gradient and exact adjoint of the density map
    wirelength   WA model, bistratal wirelength, vanilla FDA z-gradient      (Sec. III-A, IV-B)
    optimizer    mixed-size preconditioner, Nesterov step, clamp, metrics, GP loop

Parity status: the Nesterov optimiser (the paper does not describe it) is "parity unpinned":
beyond the quadratic cases its tests solve in closed form, it is pinned only by GPU-vs-oracle
parity of the same formula.  The field-gather gradient (not the derivative of any discrete
objective) is pinned by closed forms: a uniform field, and cells centred in a bin whose overlaps
are written out by hand.
"""
