"""MI355X (gfx950) implementation of the LBRMT time step.

The lattice Boltzmann reference map technique (Sun & Rycroft) couples a D2Q9
lattice Boltzmann fluid to neo-Hookean solids tracked by a reference map on one
fixed grid.  The step runs in hand-written HIP kernels behind the C ABI of
``include/lbrmt.h`` (``liblbrmt.so``); ``lbrmt`` is its thin Python binding.
"""
from .lbrmt import (Batch, LBRMTError, Sim, lib, lbrmt_add_solids, lbrmt_autotune,  # noqa: F401
                    lbrmt_band_nodes, lbrmt_batch_autotune, lbrmt_batch_create,
                    lbrmt_batch_destroy, lbrmt_batch_get_option, lbrmt_batch_init,
                    lbrmt_batch_member, lbrmt_batch_set_option, lbrmt_batch_size,
                    lbrmt_batch_step, lbrmt_batch_workspace_bytes,
                    lbrmt_create, lbrmt_debug_poke, lbrmt_get_option, lbrmt_set_option, lbrmt_destroy, lbrmt_diag, lbrmt_init,
                    lbrmt_kernel_time, lbrmt_load_state, lbrmt_read_force, lbrmt_read_macro,
                    lbrmt_read_populations, lbrmt_read_refmap, lbrmt_read_stress,
                    lbrmt_save_state, lbrmt_set_timing, lbrmt_state_bytes, lbrmt_step,
                    lbrmt_step_count, lbrmt_validate, lbrmt_workspace_bytes, make_grid_desc,
                    make_solid_desc)
