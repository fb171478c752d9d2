"""Algorithmic work of the convective right-hand side, for roofline figures.

Flops are those of the algorithm as implemented (rank-structured projections,
one-division WENO5-JS), counted as 1 per add, subtract, multiply, divide,
square root, abs or max (a fused multiply-add counts 2).  Bytes are the
algorithmic HBM traffic: every input read once, every output written once.

Per face of one direction, N species (count of the operations in the face
routine, step by step):
  Roe state and thermo at the averaged T          34 N +  36
  per-cell projection scalars and LLF speeds       18 N + 180
  acoustic pair (splitting 150, 4 WENO 276, sums 4)        430
  tangential pair (splitting 96, 4 WENO 276, sums 2)       374
  species fields (splitting 60, 2 WENO 138, rest 8) 206 N
  1 / Gamma and back-projection of momentum and energy      18
  -> F(N) = 258 N + 1038 flops per face   (one WENO5-JS = 69 flops)
plus the flux difference 2 (N + 4) per cell and direction.
"""

WENO_FLOPS = 69


def face_flops(ns):
    return 258 * ns + 1038


def sweep_flops_per_cell(ns):
    """one direction: one face (the cell's left face; the extra face per row
    is counted in `sweep_flops`) plus the flux difference of N + 4 fields"""
    return face_flops(ns) + 2 * (ns + 4)


def sweep_flops(ns, n, direction):
    """flops of one sweep launch over a grid n = (nx, ny, nz)"""
    nx, ny, nz = n
    cells = nx * ny * nz
    faces = cells + cells // n[direction]
    return faces * face_flops(ns) + cells * 2 * (ns + 4)


def rhs_flops_per_cell(ns, active=3):
    return active * sweep_flops_per_cell(ns)


def rhs_bytes_per_cell(ns):
    """read U, write rhs (FP64, N + 4 fields)"""
    return 16 * (ns + 4)


def sweep_bytes_per_cell(ns, first):
    """a sweep reads U (N + 4 fields) and the primitives T, p, c, 1/rho and
    writes rhs (the first sweep) or reads and writes it (the others)"""
    nv = ns + 4
    return 8 * (nv + 4) + (8 * nv if first else 16 * nv)


def _footprint(n, direction):
    """cells a sweep's stencils read: the interior widened by three ghost
    layers along the sweep direction"""
    m = list(n)
    m[direction] += 6
    return m[0] * m[1] * m[2]


def sweep_bytes(ns, n, direction, first=True, precision="fp64", fused_stage=False):
    """algorithmic bytes of one sweep launch: U (N + 4 fields) and the four
    primitives of every cell its stencils read, once (FP32 copies in the
    mixed path), and the residual of every interior cell written once (read
    as well when accumulated; FP32 differences in the mixed path).  With
    fused_stage (the mixed x sweep of an RK3 step, which finishes the stage
    itself) the residual is not written; instead every interior value reads
    Uin, the other two directions' residuals and, in two of the three
    stages, U0, and writes Uout (FP64 state)"""
    nv = ns + 4
    cells = n[0] * n[1] * n[2]
    word = 4 if precision == "mixed" else 8
    stencil = word * (nv + 4) * _footprint(n, direction)
    if fused_stage:
        return stencil + nv * cells * (8 + 2 * word + 8 + 8 * 2 / 3)
    return stencil + (word if first else 2 * word) * nv * cells


def stage_flops(ns, n):
    """the stage sum of Eq. 16 per interior value: three adds of the
    residuals, h L + Uin, and a U0 + b v"""
    return (ns + 4) * n[0] * n[1] * n[2] * 7


def vjp_bytes_per_cell(ns):
    """the whole RHS VJP, algorithmic: read U and the residual cotangent,
    write the state cotangent (N + 4 fields each), read T"""
    return 24 * (ns + 4) + 8


def vjp_sweep_bytes(ns, n, direction):
    """one direction of the face VJP: U and the primitives over the stencil
    footprint, the residual cotangent, and the read-modify-write of the state
    cotangent and of the three per-cell cotangents (p, T, rho)"""
    nv = ns + 4
    cells = n[0] * n[1] * n[2]
    return 8 * (nv + 4) * _footprint(n, direction) + 8 * nv * cells + 16 * (nv + 3) * cells


# Operations per face of the face VJP as implemented (the forward recomputed,
# then the backward), counted with rocprofv3's per-type VALU counters on one
# launch group of each direction at 256^3, nine species: 64 x (adds +
# multiplies + transcendentals + 2 x fused multiply-adds) of the arithmetic
# type over the group's faces (profiles/vjp_nine_species_sbi_256.md; the
# y/z figure from the group whose grid holds no idle threads).  Measured at
# nine species only: other species counts return None.
VJP_FACE_OPS = {("fp64", 9): (10178, 10226, 10226), ("mixed", 9): (10324, 10360, 10360)}

# Operations per face of the forward sweeps as executed, counted the same way
# (x sweep, nine species): FP64 3985, FP32 4155 -- about 19 % above the
# algorithmic count F(9) = 3360 of face_flops, for the divide and square-root
# sequences (counted once in F) and the rolled species loops, which
# evaluate e_s(T~) three times per species.
EXECUTED_FACE_OPS = {("fp64", 9): 3985, ("mixed", 9): 4155}


def vjp_face_flops(ns, precision="fp64", direction=0):
    c = VJP_FACE_OPS.get((precision, ns))
    return None if c is None else c[direction]


def vjp_sweep_flops(ns, n, direction, precision="fp64"):
    f = vjp_face_flops(ns, precision, direction)
    if f is None:
        return None
    cells = n[0] * n[1] * n[2]
    return f * (cells + cells // n[direction])


def rk3_step_bytes_per_cell(ns):
    """one fused-free RK3 step, algorithmic: 3 x (RHS read U + write L) plus
    3 stage updates (read U^n, U^(k-1), L; write U^(k))"""
    nv = ns + 4
    return 3 * 16 * nv + 3 * 32 * nv


SIMDS = 1024          # 256 compute units x 4 SIMDs
CLOCK_HZ = 2.4e9      # peak engine clock

PEAK = {
    "hbm_GBs": 8000.0,
    "fp64_vector_TFLOPs": 78.6,
    "fp32_vector_TFLOPs": 157.3,
}
