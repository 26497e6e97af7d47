"""MI355X (gfx950) implementation of the linearised polarised PRD transfer
operator and its GMRES solve; see include/trap.h for the C ABI."""
from .trap import Context, TrapError, load_library, footprint, TRAP_FP64, TRAP_FP32

__all__ = ["Context", "TrapError", "load_library", "footprint", "TRAP_FP64", "TRAP_FP32"]
