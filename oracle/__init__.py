"""FP64 CPU oracle for the SSPRK2-SE / SSPRK3-SE split-explicit step.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, reference
implementation that the HIP library is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the product path (``paper_2105_13484_amd``) never does, and the
oracle never imports the product path.  The two share nothing except the
seeded input generators in ``synthetic/``.

Source: R. Lan, L. Ju, Z. Wang, M. Gunzburger, P. Jones, "High-Order Multirate
Explicit Time-Stepping Schemes for the Baroclinic-Barotropic Split Dynamics in
Primitive Equations" (arXiv 2105.13484).

* ``trisk``     -- horizontal operators on the TRiSK C-grid.  The paper takes
                   them from MPAS-Ocean without stating them (Section 5
                   opening); this module states the standard TRiSK forms.
* ``layered``   -- the layered equations of Section 2 (vertical operators,
                   hydrostatic pressure, z-star vertical velocity, the
                   groupings T^u, D^u, T^h, the split BBspl, the Laplacian or
                   biharmonic horizontal viscosity, the tracer equation and
                   the linear EOS) and the vertical diffusion solve of
                   Algorithm 2.
* ``ssprk_se``  -- Section 3: Algorithms 1 and 2 (Baroclinic_FEuler and its
                   vertical-mixing form), Algorithms 3 and 4 (barotropic
                   SSPRK2/3 substepping), Interp_2 / Interp_3, the SSPRK2-SE
                   and SSPRK3-SE steps with the tracer stages, and the
                   flux-form SSH reconciliation of Section 3.4.

Everything is FP64 NumPy with whole-array operations; column sums over the
layers are correctly rounded (``layered.colsum``), so no particular addition
order is built in.

The discrete forms of the nonlinear terms (pressure gradient in tilted
layers, z-star vertical velocity, vertical boundary conditions, vorticity
flux, barotropic (zeta + H) at edges) are fixed by the readings stated in the
docstrings of these modules, not by numbers in the paper.  They are pinned by
exact properties the readings do not assume (closed forms of the pressure
gradient, z-star proportional stretching, the column budget of the vertical
fluxes, the layer-sum identity at edges) and, for the vorticity flux, by
energy neutrality and second-order consistency with the continuous term.
"""
from . import trisk, layered, ssprk_se  # noqa: F401
