"""FP64 CPU oracle for the grid-Poisson SDF reconstruction.

TEST INFRASTRUCTURE.  This package is a plain, slow, deliberately unoptimised
statement of what the reconstruction computes, written from the paper
(Warp-Geo, arXiv 2609.20964, Sec. 2.3-2.5) step by step in float64.  Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the product library never does, and the two share no code.

Modules
-------
discretize  grid, point binning, 27-cell splat weights, normal field V,
            divergence b, the 7-point operator and its exact DCT solve,
            trilinear interpolation, iso-value.
surface     Marching Cubes by a run-time rule, brute-force mesh distance,
            sign, SDF on grid nodes, sampling of SDF and normals.
adjoint     the hand-derived transposes of every linear piece and the
            reverse pass of the whole chain.
pipeline    forward / backward of the whole chain and the frozen-stencil
            finite-difference protocol.
galerkin    the Galerkin system with exact quadrature (Eq. 21, 26): the
            27-point stiffness, the consistent right-hand side, FP64 CG.
domain      grids over a box or a cloud's bounding box at density d.
normals     D-PCA normals (Eq. 1-6) and parity orientation with
            finite-radius detection and the refinement (Eq. 7-14, Sec. 2.2).
native      ctypes loader of the small C module (csrc/mcdist.c).

Conventions: "grid units" put cell centre (i,j,k) at (i,j,k); world
x = lo + (u + 1/2) h.  Grid scalars are numpy arrays indexed [k, j, i]
(x fastest in memory); vectors are [3, nz, ny, nx].
"""
