"""Plain CPU oracle for the dynamic mesh-Gaussian update (float64 unless stated).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
library (paper_2606_00444_amd) and never imports it; both sides read the same
seeded inputs from the `synth` package.

What each module follows (the paper is "Real-Time Physics Simulation with
Dynamic Mesh-Gaussian Reconstructions", arXiv 2606.00444):

* frame      frame index k = floor(t * f_recon) and the O(N_v) vertex-buffer
             copy (Sec. 3.3 MaGS paragraph; Sec. 3.4 per-frame steps 1-2).
* gaussians  face-bound Gaussians re-posed from their triangle: barycentric mean,
             triangle-frame rotation, covariance (Sec. 3.2 dual representation;
             the paper gives no binding formula, so the reading is ours and is
             pinned only by invariants - parity of the formula itself is unpinned).
* morton     30-bit Morton codes of face centroids defined in IEEE binary32, and
             the stable sort (acceleration structure built once from the template
             faces, Sec. 3.4 Initialization; LBVH construction after Karras 2012).
* lbvh       binary radix tree over the sorted codes (Karras 2012) and its bounds:
             refit = recompute every box on the fixed tree (Sec. 3.4: structures
             built from F_0 are reused for all frames; O(N_v) per frame).
* closest    closest point on a triangle (Ericson 2005, Voronoi regions) and on a
             mesh: NearestSurface with barycentric interpolation (Sec. 3.3, Eq. 2),
             read as the single nearest face (k = 1), with the winning face's unit
             normal computed on demand (Sec. 3.4 step 3).
* losses     mean squared point-to-mesh distance, two-sided Chamfer distance
             (Sec. 4.2 uses CD as a metric without a formula: squared distances,
             means, both directions, no factor 1/2), and their gradients with
             respect to the template vertices, through the binding.
* adam       Adam (Kingma & Ba 2015) with torch.optim.Adam's update order.
* knn        k-NN weighted surface projection (the NearestSurface variant of Sec. 3.3;
             k and weights unstated: k nearest faces, inverse-distance weights).
* sdf        index signed-distance grid (the SDF of Sec. 3.4): nearest template faces
             stored per node, signed distances recomputed per frame, trilinear sampling.
* contact    sphere-mesh contact step from on-demand face normals (collision response
             for the falling-sphere simulation of Sec. 4.1; the engine is out of scope).
* tracking   temporal correspondence tracking (Sec. 3.3, Eq. 1): closest points
             carried frame to frame, re-anchored to the template projection.
"""

from . import frame, gaussians, morton, lbvh, closest, losses, adam, tracking, knn, sdf, contact  # noqa: F401
