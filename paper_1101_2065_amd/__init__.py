"""MI355X-native screened Coulomb interaction W(omega) for LCAO GW.

Library: libgw.so (HIP, gfx950), C ABI in include/gw.h; Python binding in
paper_1101_2065_amd.gw (import it explicitly: it loads the built library and
raises if it is missing).
"""
__all__ = ["gw"]
