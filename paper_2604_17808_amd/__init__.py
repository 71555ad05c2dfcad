"""frntt: BN254-Fr number-theoretic transforms on AMD MI355X (gfx950).

The transforms run in libfrntt.so (hand-written HIP kernels behind a C ABI,
declared in include/frntt.h). This package only marshals arguments to it;
see ``paper_2604_17808_amd.frntt``.
"""
from .frntt import (FWD, INV, COSET, COSET_INV, ALGO_AUTO, ALGO_BUTTERFLY, ALGO_FOURSTEP_MFMA,
                    FrnttError, Context, Server, RnsField, lib, library_path, rns_moduli, RNS_Q_WORDS,
                    RNS_P_WORDS, FIELD_377, FIELD_753, msm_window, msm_workspace_bytes)

__all__ = ["FWD", "INV", "COSET", "COSET_INV", "ALGO_AUTO", "ALGO_BUTTERFLY",
           "ALGO_FOURSTEP_MFMA", "FrnttError", "Context", "Server", "lib", "library_path",
           "rns_moduli", "RNS_Q_WORDS", "RNS_P_WORDS", "RnsField", "FIELD_377", "FIELD_753",
           "msm_window", "msm_workspace_bytes"]
