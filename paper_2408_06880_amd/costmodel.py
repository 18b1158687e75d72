"""The paper's analytic byte and memory models (host arithmetic only).

Memory accesses per cell and time step follow the access tables of the AA
section (Tables "Memory accesses CPU" and "Memory accesses GPU"); memory
footprints follow the memory equation of the single-node comparison and its
AA form in the AA section.  B_pdf and B_idx are bytes per stored PDF and per
index-list entry.  The reduction of AA over pull is 1 - AA / Pull, the
definition the tables use (the inline formula of the AA section has the
ratio inverted).
"""

OTHER_FIELDS = 5   # velocity (3), density (1), flag (1), each at B_pdf


def accesses(q, b_pdf, b_idx, scheme, sparse, cpu=False):
    """Bytes moved per cell update.  Pull on a CPU pays a write-allocate
    read of the destination (3Q PDF accesses); a GPU does not (2Q).  Sparse
    kernels add the index-list: every step for pull, every second step for
    AA (only the odd step propagates)."""
    if scheme not in ("pull", "aa"):
        raise ValueError(f"scheme must be 'pull' or 'aa' (got {scheme!r})")
    pdf = (3 if (cpu and scheme == "pull") else 2) * q * b_pdf
    if not sparse:
        return pdf
    return pdf + (q - 1) * b_idx * (1.0 if scheme == "pull" else 0.5)


def aa_reduction(q, b_pdf, b_idx, sparse, cpu=False):
    """Relative saving of AA over pull in bytes moved, 1 - AA / Pull."""
    return 1.0 - (accesses(q, b_pdf, b_idx, "aa", sparse, cpu) /
                  accesses(q, b_pdf, b_idx, "pull", sparse, cpu))


def aa_step_bytes(q, b_pdf, b_idx=4):
    """Bytes of the sparse AA odd step, the even step, and their mean (the
    GPU table's AA entry): the odd step reads the index-list, the even one
    does not."""
    odd = 2 * q * b_pdf + (q - 1) * b_idx
    even = 2 * q * b_pdf
    return odd, even, 0.5 * (odd + even)


def memory(n_cells, phi, q, b_pdf, b_idx, scheme, sparse, other_fields=OTHER_FIELDS):
    """Device bytes of a solve over n_cells box cells of porosity phi: two
    PDF arrays for pull, one for the in-place AA pattern; the index-list and
    the other fields; sparse structures store fluid cells only."""
    lists = 2 if scheme == "pull" else 1
    per_cell = lists * q * b_pdf + other_fields * b_pdf
    if sparse:
        return n_cells * phi * (per_cell + (q - 1) * b_idx)
    return n_cells * per_cell


def aa_memory_saving(q, b_pdf, b_idx):
    """Saving of the sparse AA footprint over sparse pull."""
    return 1.0 - memory(1, 1.0, q, b_pdf, b_idx, "aa", True) / memory(1, 1.0, q, b_pdf, b_idx,
                                                                        "pull", True)


def memory_break_even(q, b_pdf, b_idx, scheme="pull"):
    """Porosity below which the sparse structure needs less memory than
    the dense one (same scheme on both)."""
    return memory(1, 1.0, q, b_pdf, b_idx, scheme, False) / memory(1, 1.0, q, b_pdf, b_idx,
                                                                   scheme, True)


def perf_break_even(q, b_pdf, b_idx, scheme="pull"):
    """Porosity below which a memory-bound sparse kernel updates fluid cells
    faster than a dense one that sweeps every box cell: the ratio of bytes
    per cell update, dense over sparse (GPU accesses)."""
    return accesses(q, b_pdf, b_idx, scheme, False) / accesses(q, b_pdf, b_idx, scheme, True)
