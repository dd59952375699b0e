"""Record encoding used by the trace generators (the input format, no analysis).

One event is four little-endian uint32 words ``(addr, tid, meta, aux)``:
  addr  4-byte word address (WBAR: barrier id; FENCE / BAR: 0)
  tid   block * threads_per_block + thread_in_block
  meta  kind (bits 0-3) | scope << 4 | space << 6; bits 7-31 zero
  aux   WBAR: lane mask; otherwise an opaque site id
"""
KIND = {"R": 0, "W": 1, "A": 2, "F": 3, "BAR": 4, "WBAR": 5, "ACQ": 6, "REL": 7}
SCOPE = {"BLK": 0, "-": 0, "DEV": 1, "SYS": 2}
SPACE = {"G": 0, "S": 1}


def make_meta(kind: int, scope: int = 0, space: int = 0) -> int:
    return (kind & 15) | ((scope & 3) << 4) | ((space & 1) << 6)
