"""MI355X (gfx950) library for adjoint-state wave imaging with randomized trace
estimation (Louboutin & Herrmann): forward and adjoint finite-difference
sweeps that compress the wavefield history on the fly against r random probe
vectors (Eq. 3), the probed imaging condition, and the probed FWI gradient.

The work runs in librtm.so (HIP kernels behind a C ABI, include/rtm.h); this
package is its thin Python binding.  Importing it does not load the library;
the first call does, and fails loudly if the library has not been built.
"""
from .api import (Plan, PlanSpec, RtmError, bar_index, cfl_bound, fwi_gradient,  # noqa: F401
                  rtm_adjoint_probe,
                  rtm_dot, rtm_forward_probe, rtm_image, set_stencil_variant,
                  profile_enable, profile_read, rtm_bar_to_rows,
                  fwi_gradient_exact, exact_workspace_bytes,
                  autotune_stencil, set_stencil_blocks, Batch,
                  rtm_tti_forward_probe, rtm_tti_adjoint_probe, fwi_gradient_tti,
                  set_exact_fused, set_tti_shape, set_tti_blocks, rf_workspace_bytes, rtm_sketch,
                  rtm_orthonormalize, fwi_gradient_rf, rtm_offset_gathers,
                  stream_status, rtm_forward_probe_range, fwi_gradient_noalloc,
                  rtm_residual, tti_spectral_radius, set_stencil_alternate,
                  set_probe_nt, set_probe_grid, set_graph)
