/*
 * ftn.h -- C ABI of the MI355X fermionic tensor contraction library.
 *
 * Implements the pairwise operations of fermionic tensor networks on
 * symmetry-blocked (Abelian) tensors as described in "Fermionic tensor
 * network contraction for arbitrary geometries" (Gao et al.):
 *   - symmetric tensors with +/- leg labels and total charge (Sec. II.A,
 *     Eq. symmetryrule), with parity and leg order (Sec. II.B);
 *   - fermionic transposition (Eq. transposition) and contraction
 *     (Eq. standardcontract) under the globally ordered (Sec. II.D) and the
 *     locally ordered (Sec. II.E) conventions;
 *   - arrow reversal as a bond parity tensor (Sec. II.E, Fig. 3b) and index
 *     fusion with its three parity contributions (Sec. IV.A);
 *   - bond compression by truncated SVD with the chi largest singular values
 *     kept over all symmetry blocks (Sec. II.A), used by approximate
 *     contraction (Fig. 1b, Sec. III);
 *   - contraction of a whole network along a given pairwise path.
 *
 * Conventions shared by every call
 *   - Return value: FTN_OK (0) or a negative FTN_E* code. A message for the
 *     last error of the calling thread is returned by ftn_last_error().
 *     Calls never throw and never abort the process.
 *   - Charges: every charge is a pair of int32 (q0, q1). Z2 uses q0 in {0,1}
 *     and q1 = 0; U(1) uses q0 and q1 = 0; U(1)xU(1) uses both (n_up, n_dn).
 *     Fermion parity is (q0 + q1) mod 2 (an odd U(1) charge is odd).
 *   - Dual flags: 0 = '+' (outgoing), 1 = '-' (incoming). In the local
 *     convention an arrow runs from the '+' end to the '-' end of a bond
 *     (the default labelling of Sec. IV.B).
 *   - Sectors of a leg are given in strictly ascending charge order
 *     (lexicographic for U(1)xU(1)); dims must be positive.
 *   - Blocks: the allowed sector-index keys in lexicographic order; inside a
 *     block, entries are row-major over the legs. The data buffer holds the
 *     blocks back to back in that order (no padding).
 *   - Handles: ftn_tensor_t and ftn_net_t are opaque and library-owned.
 *     Input handles are borrowed and never modified. Every handle written to
 *     an `out` argument is new, owned by the caller and released with
 *     ftn_tensor_free / ftn_net_free.
 *   - Device memory: tensor data lives in device memory of the current HIP
 *     device, allocated by the library (its caching allocator: blocks freed
 *     on a stream are reused in that stream's order and kept until the
 *     process ends or an allocation fails; or the allocator registered with
 *     ftn_set_allocator).
 *   - Streams: work is enqueued on the given stream. Calls that must know a
 *     data-dependent size (block counts of a new structure, the dims kept by
 *     a truncation) synchronise that stream before returning. A tensor's
 *     memory is released in the order of the stream that created it, so that
 *     stream must outlive the tensor, and a tensor read by work on another
 *     stream must not be freed before that work has completed (synchronise
 *     the other stream, or make the creating stream wait on it, first). The
 *     library's own shared state (block structures, cached plans) may be
 *     used from several streams at once.
 *   - Threads: a handle must not be used by two threads at once.
 */
#ifndef FTN_H
#define FTN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* ftn_stream_t; /* a hipStream_t; NULL = default */

enum {
  FTN_OK = 0,
  FTN_EINVAL = -1,   /* bad argument: shape, permutation, axis, null pointer */
  FTN_ECHARGE = -2,  /* contracted legs with equal duals, or one charge with
                        different dims on the two sides of a bond */
  FTN_ENOMEM = -3,   /* device allocation failed */
  FTN_EHIP = -4,     /* a HIP runtime call failed */
  FTN_ENOCONV = -5,  /* an iterative decomposition did not converge */
  FTN_ENOTSUP = -6   /* combination not supported (e.g. dtype mix) */
};

typedef enum { FTN_Z2 = 0, FTN_U1 = 1, FTN_U1xU1 = 2 } ftn_sym;
typedef enum { FTN_F64 = 0, FTN_F32 = 1 } ftn_dtype;
typedef enum { FTN_LOCAL = 0, FTN_GLOBAL = 1 } ftn_conv;
/* arithmetic of the block-pair GEMMs: FP64 MFMA, FP32 MFMA, or split-BF16
   compensated products (hi*hi + hi*lo + lo*hi) on BF16 MFMA with FP32
   accumulation; the two FP32 forms require FTN_F32 tensors. */
typedef enum { FTN_GEMM_F64 = 0, FTN_GEMM_F32 = 1, FTN_GEMM_BF16X3 = 2 } ftn_gemm;

typedef struct ftn_tensor* ftn_tensor_t;
typedef struct ftn_net* ftn_net_t;

/* Last error message of the calling thread ("" if none). Owned by the
   library, valid until the next failing call on the same thread. */
const char* ftn_last_error(void);

/* Library version string. */
const char* ftn_version(void);

/* Optional external device allocator (e.g. a framework's caching pool).
   alloc(bytes, stream, ctx) returns device memory or NULL; free(ptr, stream,
   ctx) releases it. Pass NULLs to restore the built-in caching allocator. */
int ftn_set_allocator(void* (*alloc_fn)(size_t, ftn_stream_t, void*),
                      void (*free_fn)(void*, ftn_stream_t, void*), void* ctx);

/* ---------------------------------------------------------------------------
 * Tensors (Sec. II.A Eq. symmetryrule; Sec. II.B parity and leg order)
 * ------------------------------------------------------------------------ */

/* Create a symmetric fermionic tensor.
   ndim legs (0 <= ndim <= 16); leg i has nsect[i] sectors; the sectors of
   all legs are concatenated in `charges` (2 int32 per sector) and
   `sect_dims` (int64 per sector); dual[i] in {0,1}; total_charge = 2 int32.
   The allowed blocks are enumerated on the device (lexicographic keys).
   If `src` is non-NULL it is a device buffer holding the block data in the
   documented layout (as many entries as the tensor has), which is copied;
   otherwise the data are zero. */
int ftn_tensor_create(ftn_sym sym, ftn_dtype dtype, int ndim, const int32_t* nsect,
                      const int32_t* charges, const int64_t* sect_dims,
                      const uint8_t* dual, const int32_t* total_charge,
                      const void* src, ftn_stream_t stream, ftn_tensor_t* out);

/* Same structure arguments; the tensor's block data are the caller's device
   buffer dev_data (the documented layout, as many entries as the tensor
   has), used in place without a copy: the buffer is borrowed, must stay
   alive and unchanged while the handle or any tensor sharing its data (a
   network built from it) is in use, and is never freed by the library. */
int ftn_tensor_wrap(ftn_sym sym, ftn_dtype dtype, int ndim, const int32_t* nsect,
                    const int32_t* charges, const int64_t* sect_dims, const uint8_t* dual,
                    const int32_t* total_charge, void* dev_data, ftn_stream_t stream,
                    ftn_tensor_t* out);

/* Same structure arguments; the data are gathered on the device from a
   dense row-major array `dense` (device memory, same dtype as the tensor)
   whose leg index spaces are the leg's sectors concatenated in order.
   Entries outside allowed blocks are ignored. */
int ftn_tensor_from_dense(ftn_sym sym, ftn_dtype dtype, int ndim, const int32_t* nsect,
                          const int32_t* charges, const int64_t* sect_dims,
                          const uint8_t* dual, const int32_t* total_charge,
                          const void* dense, ftn_stream_t stream, ftn_tensor_t* out);

/* Scatter the blocks into a dense row-major device array (zeros elsewhere).
   `dense` must hold prod(leg sizes) entries of the tensor's dtype. */
int ftn_tensor_to_dense(ftn_tensor_t t, void* dense, ftn_stream_t stream);

/* Structure queries. Pointers returned stay valid while the handle lives.
   keys: nblocks*ndim int32 sector indices; offsets: nblocks+1 int64 entry
   offsets; shapes: nblocks*ndim int64. */
int ftn_tensor_info(ftn_tensor_t t, int* sym, int* dtype, int* ndim, int64_t* nblocks,
                    int64_t* size, int32_t total_charge[2]);
int ftn_tensor_blocks(ftn_tensor_t t, const int32_t** keys, const int64_t** offsets,
                      const int64_t** shapes);
/* Leg i: number of sectors, charges (2 int32 each), dims, dual. */
int ftn_tensor_leg(ftn_tensor_t t, int leg, int32_t* nsect, const int32_t** charges,
                   const int64_t** dims, uint8_t* dual);
/* Device pointer of the block data (valid while the handle lives). */
int ftn_tensor_data(ftn_tensor_t t, void** dev_ptr);
/* Copy the block data into `dst` (device memory, size entries). */
int ftn_tensor_copy_data(ftn_tensor_t t, void* dst, ftn_stream_t stream);
/* Convert to another dtype (FP64 <-> FP32, round to nearest even). */
int ftn_tensor_cast(ftn_tensor_t t, ftn_dtype dtype, ftn_stream_t stream, ftn_tensor_t* out);
/* out = alpha * t (alpha applied in the tensor's dtype). */
int ftn_tensor_scale(ftn_tensor_t t, double alpha, ftn_stream_t stream, ftn_tensor_t* out);
/* out = alpha * x + y (x and y of one structure and dtype), e.g. to combine
   the gradients of several networks. */
int ftn_tensor_axpy(double alpha, ftn_tensor_t x, ftn_tensor_t y, ftn_stream_t stream, ftn_tensor_t* out);
int ftn_tensor_free(ftn_tensor_t t);

/* ---------------------------------------------------------------------------
 * Unary fermionic operations
 * ------------------------------------------------------------------------ */

/* Fermionic transposition, Eq. (transposition): new leg t is old leg
   perm[t]; every block is multiplied by (-1)^kappa with kappa the sum of
   p_i p_j over the pairs of legs whose order the permutation inverts. */
int ftn_ftranspose(ftn_tensor_t a, const int32_t* perm, ftn_stream_t stream,
                   ftn_tensor_t* out);

/* Reverse the dual of one leg (charges conjugated, sector order updated).
   with_sign = 1 multiplies by (-1)^{p} of the leg's sector: reversing an
   arrow is a bond parity tensor (Sec. II.E, Fig. 3b), so a bond is reversed
   by flipping both ends, one of them with the sign. with_sign = -1 means
   "sign iff the leg was '-'", the library's convention for that one end. */
int ftn_flip_dual(ftn_tensor_t a, int leg, int with_sign, ftn_stream_t stream,
                  ftn_tensor_t* out);

/* Hermitian conjugate of one tensor (Sec. II.D, Fig. 4a: the bra reverses
   the order of the tensors and the indices of each): legs in reverse order,
   duals flipped with charge labels kept, total charge negated, entries
   conjugated (real here). Reversing the legs is a relabelling and carries no
   sign. */
int ftn_dagger(ftn_tensor_t a, ftn_stream_t stream, ftn_tensor_t* out);

/* Fuse legs[0..nlegs) (in this order) into one leg placed where legs[0]
   stood among the remaining legs (Sec. IV.A): (1) fermionic transposition
   making them adjacent; (2) legs whose dual differs from legs[0]'s are
   flipped (local: ftn_flip_dual with with_sign = -1; global: no sign);
   (3) the reversal sign sum_{s<t} p_s p_t of reading the fused modes in
   reverse order is applied when the fused leg is '-' (local) or when
   rev = 1 (global; the later of the two tensors sharing the bond).
   Fused sectors: distinct sums of the component charges (ascending); inside
   one, component key combinations in lexicographic order, concatenated. */
int ftn_fuse(ftn_tensor_t a, int nlegs, const int32_t* legs, ftn_conv conv, int rev,
             ftn_stream_t stream, ftn_tensor_t* out);

/* Adjoint of ftn_fuse: for a cotangent dout of the fused tensor (its
   structure), the cotangent da of a (new handle, structure of a). Fusion
   moves every entry of a to one entry of the output with a sign, so da reads
   each entry back with the same sign. */
int ftn_fuse_backward(ftn_tensor_t a, int nlegs, const int32_t* legs, ftn_conv conv, int rev,
                      ftn_tensor_t dout, ftn_stream_t stream, ftn_tensor_t* da);

/* ---------------------------------------------------------------------------
 * Contraction, Eq. (standardcontract)
 * ------------------------------------------------------------------------ */

/* C = sum^F over the pairs (axes_a[t], axes_b[t]) of A and B, output legs =
   free legs of A in order ++ free legs of B in order, s(C) = s(A) + s(B).
   Contracted legs must have opposite duals (FTN_ECHARGE otherwise); a charge
   present on one side only contributes nothing. Sign per matched block pair:
   Koszul sign of A -> free(A) ++ axes_a, of B -> axes_b ++ free(B), the
   reversal sign sum_{s<t} p_s p_t of pairing in list order, and with
   FTN_LOCAL the bond parity (-1)^{p} of every bond whose end on A is '+'
   (contracted against its arrow, Eq. fermionictn2). FTN_GLOBAL is F(AB)
   with A immediately left of B (Sec. II.D). The work runs as signed permutes
   into per-charge fused matrices and one grouped MFMA GEMM. A and B must
   have the same dtype; gemm selects the arithmetic (see ftn_gemm). */
int ftn_ftensordot(ftn_tensor_t a, ftn_tensor_t b, int naxes, const int32_t* axes_a,
                   const int32_t* axes_b, ftn_conv conv, ftn_gemm gemm,
                   ftn_stream_t stream, ftn_tensor_t* out);

/* Adjoint (reverse-mode derivative) of ftn_ftensordot. The contraction is
   bilinear in A and B (Eq. standardcontract), so for a cotangent dC of C:
   dA = sum over blocks of the same signed pairing with dC and B (the free
   legs of B contracted), dB likewise with A and dC, with exactly the signs of
   the forward call. dc must have the structure of the forward output (same
   legs, duals and total charge as ftn_ftensordot(a, b, ...) returns); da and
   db are new tensors with the structures of a and b. Arguments as in
   ftn_ftensordot; runs as the forward permutes, one gather of dC into the
   per-charge fused matrices, two grouped GEMMs (dA~ = dC B~^T,
   dB~ = A~^T dC) and the permutes run backwards. */
int ftn_ftensordot_backward(ftn_tensor_t a, ftn_tensor_t b, ftn_tensor_t dc, int naxes,
                            const int32_t* axes_a, const int32_t* axes_b, ftn_conv conv,
                            ftn_gemm gemm, ftn_stream_t stream, ftn_tensor_t* da,
                            ftn_tensor_t* db);

/* Allocation-free form of ftn_ftensordot, for callers that cannot allocate
   device memory (code under HIP graph capture, tight serving loops, harnesses
   that forbid allocation). Same arguments and result as ftn_ftensordot, but
   the output blocks are written to out_data (device memory of the current
   device, out_size entries of the tensors' dtype, in the block layout of the
   output structure that ftn_ftensordot returns for these operands), and the
   temporaries (fused matrices, split-K workspace) live in a fixed 64 MiB
   device array that the library holds on each GPU until the process ends.
   No device memory is allocated or freed, so the contraction plan must be
   cached: call ftn_ftensordot once with operands of the same structures,
   axes, convention and GEMM form first (FTN_ENOTSUP otherwise).
   FTN_EINVAL if out_size differs from the output's size or if the
   temporaries exceed 64 MiB. Every call on one GPU uses that GPU's array:
   calls that overlap in time on one GPU (other streams or threads) race and
   must be serialised by the caller; the array keeps the last call's
   contents, every entry a call reads it has written first. */
int ftn_ftensordot_noalloc(ftn_tensor_t a, ftn_tensor_t b, int naxes, const int32_t* axes_a,
                           const int32_t* axes_b, ftn_conv conv, ftn_gemm gemm,
                           ftn_stream_t stream, void* out_data, int64_t out_size);

/* ---------------------------------------------------------------------------
 * Bond compression (Sec. II.A truncated SVD; Sec. III approximate trees)
 * ------------------------------------------------------------------------ */

/* Compress the single bond between leg leg_a of A and leg leg_b of B to at
   most chi (chi >= 1): returns A', B' whose contraction over the new bond
   is the best rank-chi approximation of F(AB) across that bond, keeping the
   chi largest singular values over all charge sectors (ties: larger value,
   then lower charge, then lower index). Values not above cutoff * s_max are
   dropped (cutoff >= 0, FTN_EINVAL otherwise) and empty sectors removed.
   Bond sectors of dimension up to 128 take exact triangular factors of both
   sides (shifted Cholesky QR, three passes) and a one-sided Jacobi SVD of
   their product, which resolves singular values to about 1e-15 of the
   largest; larger sectors reach their values through Gram matrices, which
   resolve them only to ~1e-7 of the sector's largest, and there values below
   1e-6 of it count as zero. If no charge of the bond carries blocks on both
   sides, F(AB) is zero across the bond: nothing is kept and the bond leg
   of both outputs has no sector. The bond keeps its leg positions,
   duals and charge labels; only sector dims shrink. conv selects how F(AB)
   is read (as in ftn_ftensordot). FP64 arithmetic is used for the
   decomposition whatever the tensors' dtype. discarded_weight (may be NULL)
   receives the sum of the squares of the dropped singular values; svals
   (may be NULL, room for chi doubles) receives the kept values in
   descending order. Synchronises the stream. */
int ftn_compress_bond(ftn_tensor_t a, ftn_tensor_t b, int leg_a, int leg_b, int64_t chi,
                      double cutoff, ftn_conv conv, ftn_stream_t stream, ftn_tensor_t* a_out,
                      ftn_tensor_t* b_out, double* discarded_weight, double* svals,
                      int64_t* nkept);

/* Adjoint of ftn_compress_bond: for cotangents da_out, db_out of its outputs
   (structures of a_out, b_out), the cotangents da, db (structures of a, b,
   new handles) of the map (a, b) -> (a_out, b_out) computed with the same
   arguments, the number of values kept per charge held fixed. This is the
   derivative of the truncated SVD of the bond matrix C = A~ B~ per charge
   (Sec. II.A): with C = U S V^T and a_out = U_k S_k^1/2, b_out = S_k^1/2 V_k^T,
   dC = U Y V^T + (I - U U^T) G_u S_k^-1 V_k^T + U_k S_k^-1 G_v^T (I - V V^T),
   G_u = da_out S_k^1/2, G_v = db_out^T S_k^1/2, and Y the usual coupling
   matrix (s_i^2 - s_j^2)^-1 over all nonzero singular values; then
   dA~ = dC B~^T and dB~ = A~^T dC, run back through the signed permutes.
   Valid for losses unchanged by a_out -> a_out D, b_out -> D b_out with D
   diagonal +-1 (sign of each kept singular vector pair); couplings of
   singular values closer than 1e-13 s_max^2 are dropped. FP64 only
   (FTN_ENOTSUP otherwise); bond sectors of dimension up to 1024 (FTN_ENOTSUP
   for larger ones): the eigenpairs of X X^T come from Jacobi sweeps in LDS up
   to order 128 and from block Jacobi above (pairs of blocks of at most 64
   diagonalised in LDS, the whole matrix rotated by GEMMs, until the
   off-diagonal norm is at most 8 n u of the matrix's). Synchronises the
   stream. */
int ftn_compress_bond_backward(ftn_tensor_t a, ftn_tensor_t b, int leg_a, int leg_b, int64_t chi,
                               double cutoff, ftn_conv conv, ftn_tensor_t da_out, ftn_tensor_t db_out,
                               ftn_stream_t stream, ftn_tensor_t* da, ftn_tensor_t* db);

/* ---------------------------------------------------------------------------
 * Networks (Secs. II.C-II.E; Fig. 1)
 * ------------------------------------------------------------------------ */

/* A network of ntensors tensors (borrowed: the network keeps its own
   references) and nbonds bonds, bond_ends[4*i..] = (t1, l1, t2, l2).
   conv = FTN_GLOBAL: positions[t] is the global position of tensor t
   (Eq. fermionictn); the network is translated once into the locally
   ordered form (Sec. II.D: positions define a DAG): the duals of bonds
   whose '-' end sits on the later tensor are relabelled, and odd tensors
   get size-1 odd dummy legs sorted by position at the end (Sec. II.E).
   conv = FTN_LOCAL: arrows are the duals; positions (may be NULL) only fix
   the order in which dummy legs of odd tensors are sorted (default: tensor
   index). */
int ftn_net_create(int ntensors, const ftn_tensor_t* tensors, int nbonds,
                   const int32_t* bond_ends, ftn_conv conv, const int32_t* positions,
                   ftn_net_t* out);
int ftn_net_free(ftn_net_t net);

/* Contract the network along an SSA path (nsteps pairs; inputs are ids
   0..n-1, step k creates id n+k). Every step contracts all bonds the pair
   shares. With chi > 0 (approximate contraction, compression as early as
   possible, Sec. III): after each step the bonds the new tensor shares with
   one neighbour are fused into one (Sec. IV.A) and every such bond larger
   than chi is compressed with ftn_compress_bond (cutoff 1e-12). chi <= 0
   means exact. Every intermediate is rescaled by a power of two; the value
   is mantissa * 2^exp2. For a closed network the result is a scalar and
   open_out may be NULL; otherwise *open_out receives the final tensor (its
   legs are the open legs; leg_src (may be NULL, 2 int32 per leg) receives
   the (tensor, leg) each came from) scaled by 2^-exp2.
   stats (may be NULL, 8 doubles): [0] useful GEMM flops, [1] compressions,
   [2] total discarded weight, [3] near ties flagged at truncation cuts,
   [4] max intermediate entries, [5] textbook flops of the compressions
   (per bond sector: QR and LQ of the two sides with thin factors,
   4 m n^2 - 4 n^3 / 3 each, m >= n; thin SVD of the core, 14 m n^2 + 8 n^3;
   absorbing the kept vectors, 2 m r k per side), [6..7] reserved. */
int ftn_contract_network(ftn_net_t net, int nsteps, const int32_t* ssa_path, int64_t chi,
                         ftn_gemm gemm, ftn_stream_t stream, double* mantissa, int64_t* exp2,
                         ftn_tensor_t* open_out, int32_t* leg_src, double* stats);

/* Value and reverse-mode derivative of a closed network in the local
   convention (FP64 tensors, FTN_GEMM_F64; FTN_ENOTSUP otherwise): the same
   steps as ftn_contract_network (contraction, fusion, compression as early as
   possible with cutoff 1e-12, power-of-two rescaling), recorded and run
   backwards through the adjoints of contraction (Eq. standardcontract is
   bilinear), fusion (a signed permutation) and compression (the truncated-SVD
   derivative of ftn_compress_bond_backward, kept counts fixed; bond sectors up
   to 1024), each rescaling by its own power of two, and the sign of the dummy
   legs of odd tensors as a constant factor. value = mantissa * 2^exp2;
   grads[t] (ntensors new handles, structure of tensor t) holds
   d(value)/d(tensor t) * 2^-exp2. checkpoint = 0 keeps every intermediate for
   the backward pass; checkpoint = s >= 1 keeps only the tensors alive at the
   start of every s-th path step (the environments at the segment boundaries)
   and recomputes one segment at a time during the backward pass. */
int ftn_contract_network_grad(ftn_net_t net, int nsteps, const int32_t* ssa_path, int64_t chi,
                              ftn_gemm gemm, int checkpoint, ftn_stream_t stream, double* mantissa,
                              int64_t* exp2, ftn_tensor_t* grads);

/* Amplitudes <n|psi> of a fermionic tensor network state (the coefficient
   tensor of the ket network, Secs. II.D-II.E): for every sample k,
   mantissa[k] * 2^exp2[k] = Psi_{n^k} for the configuration
   n^k = configs[k * nsites + i], i = 0..nsites-1 (physical index of site i).
   sites: nsites tensors whose leg 0 is the physical leg (borrowed); the site
   order is the global order, so the coefficient has the physical legs in
   site order. bond_ends: nbonds x (site, leg, site, leg) with legs >= 1 (the
   closed network of the projected tensors; legs keep their numbering).
   Each site tensor is projected on the physical index (entries T[n_i, ...],
   computed once per distinct index), the closed network of projections is
   contracted along ssa_path (nsites-1 steps) in the local convention with
   compression to chi as ftn_contract_network does (chi <= 0: exact), and
   the sign of fixing the physical legs, (-1)^E with
   E = sum_i p(n_i) sum_{j<i} (p(T_j) + p(n_j)), is applied (the physical
   leg of site i passes the bond legs of the earlier sites). Configurations
   of the wrong total charge give mantissa 0. Samples are independent:
   nworkers host threads (1..64), each with its own HIP stream (created on
   first use and kept by the library), take them from a shared counter. Inputs must be ready on `stream`; the call returns
   when every amplitude is written (host arrays). */
int ftn_amplitudes(int nsites, const ftn_tensor_t* sites, int nbonds, const int32_t* bond_ends,
                   int nsteps, const int32_t* ssa_path, int64_t chi, ftn_gemm gemm, int64_t nsamples,
                   const int32_t* configs, int nworkers, ftn_stream_t stream, double* mantissa,
                   int64_t* exp2);

/* ---------------------------------------------------------------------------
 * Tile autotuner of the grouped GEMM (the block-pair products of every
 * contraction and the products of bond compression)
 * ------------------------------------------------------------------------ */

/* mode 0: tile shapes from the built-in heuristic (default); 1: from the
   tuning table where it has an entry for the plan's shape key (the GEMM
   form, the binary orders of the largest M, N, K and of the group count,
   symmetric and scatter flags), else the heuristic; 2: as 1, and a plan
   whose key has no entry is tuned first: every tile configuration whose
   padded tiles stay within four times the useful area, with and without
   split-K, is timed on scratch operands of the plan's extents (one warm-up,
   median of three) and the fastest is stored. Tuning allocates and
   synchronises the stream; results of different tile shapes differ only by
   rounding. The table is process-wide. */
int ftn_autotune(int mode);
/* Merge entries from / write the table to a JSON file
   ({"entries": {"<key>": [config, split, microseconds], ...}}). */
int ftn_autotune_load(const char* path);
int ftn_autotune_save(const char* path);
/* Entries in the table, keys tuned by this process, plans that took a
   stored choice (any pointer may be NULL). */
int ftn_autotune_stats(int64_t* entries, int64_t* tuned, int64_t* hits);

/* ---------------------------------------------------------------------------
 * Kernel timing (measurement support)
 * ------------------------------------------------------------------------ */

/* kernel classes reported by ftn_profile_collect */
enum {
  FTN_PROF_GEMM_F64 = 0,    /* grouped GEMM, FP64 MFMA; work = useful flops */
  FTN_PROF_GEMM_F32 = 1,    /* grouped GEMM, FP32 MFMA; work = useful flops */
  FTN_PROF_GEMM_BF16X3 = 2, /* grouped GEMM, split BF16; work = useful flops */
  FTN_PROF_PERMUTE = 3,     /* signed block permutes; work = bytes read + written */
  FTN_PROF_FACTOR = 4,      /* Cholesky / Jacobi kernels; work = textbook flops
                               (Cholesky p^3/3, triangular inverse p^3/3,
                               symmetric eigensolver with vectors 9 n^3) */
  FTN_PROF_OTHER = 5,
  /* single kernels inside classes 0 and 4, for per-kernel rooflines. Their
     time, launches and work are also counted in the class they belong to,
     except that the split-K reduction and the eigenvector kernel add time
     only (a grouped GEMM is one launch of class 0, its reduction included;
     an eigensolve's launch is its sweep kernel). */
  FTN_PROF_K_GEMM_F64_64x64 = 6,   /* k_gemm FP64, 64 x 64 tiles; work = useful flops */
  FTN_PROF_K_GEMM_F64_128x128 = 7, /* 128 x 128 tiles */
  FTN_PROF_K_GEMM_F64_256x16 = 8,  /* 256 x 16 tiles */
  FTN_PROF_K_GEMM_F64_256x32 = 9,  /* 256 x 32 tiles */
  FTN_PROF_K_GEMM_F64_16x256 = 10, /* 16 x 256 tiles */
  FTN_PROF_K_GEMM_F64_32x256 = 11, /* 32 x 256 tiles */
  FTN_PROF_K_SPLITK_F64 = 12,      /* split-K reduction, FP64; work = bytes read + written */
  FTN_PROF_K_ORTH = 13,            /* Cholesky with triangular inverse (k_orth_factor) */
  FTN_PROF_K_JACOBI = 14,          /* Jacobi sweeps, orders below 63 */
  FTN_PROF_K_JACOBI_LA = 15,       /* Jacobi sweeps, one barrier per round (orders 63..128) */
  FTN_PROF_K_JACOBI_VEC = 16,      /* eigenvector accumulation (work counted with the sweeps) */
  FTN_PROF_K_SVD_COLS = 17,        /* one-sided Jacobi SVD */
  FTN_PROF_K_SKINNY_F64 = 18,      /* tall-skinny A^T B (outputs of at most 32 x 32), FP64, with
                                      its partial-sum reduction */
  FTN_PROF_K_GEMM_F64_TALL = 19,   /* tall A B with N <= 16 and K <= 256 (A streamed once), FP64 */
  FTN_PROF_NCLASS = 20
};

/* on != 0: bracket every instrumented launch with HIP events on its stream
   (adds a little launch overhead); 0: stop. Accumulated figures are kept. */
int ftn_profile_enable(int on);
/* Per class (FTN_PROF_NCLASS entries each, any may be NULL): summed kernel
   milliseconds, launch counts, attributed work and algorithmic bytes (GEMM:
   every entry of A, B and C once; permute: bytes read + written) since the
   last collect. Synchronises the recorded events and resets the
   accumulators. */
int ftn_profile_collect(double* ms, double* count, double* work, double* bytes);

/* Device memory of the built-in caching allocator on `device` (a HIP device
   index), in bytes: `in_use` held by live buffers (tensor data, plans,
   temporaries; sizes rounded as allocated), `peak` the largest in_use since
   the last reset, `reserved` obtained from hipMalloc (in use + cached). Any
   pointer may be NULL. reset_peak != 0 then sets peak to the current in_use
   (the values returned are those before the reset).
   Memory from an external allocator and persistent tables (hipMalloc
   directly) are not counted. FTN_EINVAL for a device index out of range. */
int ftn_memory_stats(int device, int64_t* in_use, int64_t* peak, int64_t* reserved, int reset_peak);

#ifdef __cplusplus
}
#endif

#endif /* FTN_H */
