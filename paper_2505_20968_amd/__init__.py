"""MI355X (gfx950) implementation of the linearised polarised PRD transfer
operator and its GMRES solve; see include/trap.h for the C ABI."""
from .trap import (Context, TrapError, load_library, footprint, faddeeva, hip_notes, gmres_step_batch, TRAP_FP64, TRAP_FP32,
                   TRAP_PATH_AUTO,
                   TRAP_PATH_FUSED, TRAP_PATH_CHUNKED, TRAP_PRD_AD, TRAP_PRD_AA, TRAP_FORMAL_DELO_LINEAR,
                   TRAP_FORMAL_DELOPAR, TRAP_FORMAL_BESSER, TRAP_INTERP_SPLINE, TRAP_INTERP_WENO4)

__all__ = ["Context", "TrapError", "load_library", "footprint", "faddeeva", "hip_notes", "gmres_step_batch", "TRAP_FP64", "TRAP_FP32",
           "TRAP_PATH_AUTO", "TRAP_PATH_FUSED", "TRAP_PATH_CHUNKED", "TRAP_PRD_AD", "TRAP_PRD_AA",
           "TRAP_FORMAL_DELO_LINEAR", "TRAP_FORMAL_DELOPAR", "TRAP_FORMAL_BESSER", "TRAP_INTERP_SPLINE",
           "TRAP_INTERP_WENO4"]
