/*
 * zc.h -- C ABI of the MI355X (gfx950) SumCheck prover for multilinear
 * ZeroCheck over the BN254 scalar field.
 *
 * The operation is the multilinear ZeroCheck of "When Proofs Meet Hardware:
 * Comparing NTT and SumCheck in Zero-Knowledge Systems", Fig. 2 (right) and
 * Sec. 3.3 (Eq. (1)): given the MLE tables of the witness columns of a gate
 * f_M and a point r, prove sum_x f_M(x) eq_r(x) = 0 over {0,1}^mu by
 * SumCheck.  Round i sends G_i(X) = sum over x_{i+1..mu} of
 * f_M(alpha_1..alpha_{i-1}, X, x_{>i}) eq_r(...) as its d+2 values at
 * X = 0..d+1, takes alpha_i from the transcript, and folds every table
 * (Sec. 4.1).  After mu rounds the tables hold the openings at alpha.
 *
 * Conventions shared by every entry point:
 *  - Field elements at the boundary are canonical (< p), 8 x uint32
 *    little-endian limbs (= the 32-byte little-endian encoding).
 *  - Tables handed to the prover are in the library's internal form made by
 *    zc_pack: limb-planar, limb l of element j at table[l * pitch + j],
 *    pitch = 2^mu, Montgomery form.  They are opaque otherwise.
 *  - Index convention: table index b = sum_i x_i 2^(mu-i); x_1 is the most
 *    significant bit and is bound first.
 *  - Transcript: T_0 = SHA-256("ZCv1" || u32le mu || u32le gate || u32le m ||
 *    enc(r_1) .. enc(r_mu)); T_i = SHA-256(T_{i-1} || enc(G_i(0)) .. enc(G_i(d+1)));
 *    alpha_i = T_i read as a little-endian integer, mod p.
 *  - All pointers are device pointers unless stated otherwise; the caller
 *    allocates and owns every buffer.  The library allocates nothing and
 *    keeps no global state between calls; calls with distinct workspaces may
 *    run concurrently on distinct streams.
 *  - Work is enqueued on `stream` and is complete when that stream has been
 *    synchronized.  Host-side argument checks return a negative zc_status
 *    and enqueue nothing.  A failed launch returns ZC_EHIP.  Conditions the
 *    device detects (an input >= p, a stepping call out of order) are stored
 *    in the workspace and returned by zc_read_error.
 */
#ifndef ZC_H
#define ZC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ZC_OK = 0,
  ZC_EINVAL = -1,       /* bad argument (null pointer, mu out of range, bad round index) */
  ZC_EUNSUPPORTED = -2, /* unknown gate or gate parameter */
  ZC_EHIP = -3,         /* a HIP call or kernel launch failed */
  ZC_ERANGE = -4,       /* (device) an input element was >= p */
  ZC_ESTATE = -5,       /* (device) zc_round / zc_fold called out of order */
  ZC_ETOOBIG = -6,      /* the shape needs more workspace than zc_prove_static holds */
  ZC_ECLAIM = -7        /* (device, ZC_FLAG_CHECK_CLAIMS) a round failed the verifier's claim check */
} zc_status;

/* zc_shape.flags */
enum {
  /* Self-checks on the device (debug): each round checks
     G_i(0) + G_i(1) = G_{i-1}(alpha_{i-1}) (Sec. 3.4; 0 for i = 1, which a
     witness that does not satisfy the gate fails), and the proof's last step
     checks G_mu(alpha_mu) = f_M(openings) eq_r(alpha).  A failure is stored
     as ZC_ECLAIM (zc_read_error); the outputs are unchanged.  Costs a
     Lagrange evaluation per round on an otherwise idle lane. */
  ZC_FLAG_CHECK_CLAIMS = 1,
  /* The GPU is shared with other streams (e.g. several proofs at once):
     thread-per-pair round kernels are launched with up to 2048 blocks of at
     least 2 pairs a thread, instead of one generation of blocks resident for
     the whole round, so that compute units come free during a round for
     other streams' kernels.  The proof's bytes do not change; alone, a large
     proof takes a few percent longer.  zc_prove / zc_prove_pitch /
     zc_prove_static only (batches and serving size their own grids). */
  ZC_FLAG_SHARED_GPU = 2,
  /* The caller asserts that the witness satisfies the gate on the whole
     hypercube (f_M = 0 at every row), so that G_1(0) = G_1(1) = 0: round 1
     then evaluates the points X = 2..d+1 only (Sec. 3.3: every hypercube
     term of H_1(0) and H_1(1) vanishes).  For such a witness the bytes are
     those of the proof without the flag.  For any other witness the proof
     is not the honest one (its G_1(0), G_1(1) are 0).  zc_prove /
     zc_prove_pitch / zc_prove_static only; batches and serving ignore it. */
  ZC_FLAG_ASSUME_SATISFIED = 4
};

typedef enum {
  /* f = qM*a*b + qL*a + qR*b + qO*c + qC, degree 3,
     tables [a, b, c, qM, qL, qR, qO, qC] (HyperPlonk-style vanilla gate) */
  ZC_GATE_VANILLA = 0,
  /* f = s*w1*...*wm - o, degree m+1, tables [s, w1, .., wm, o], 1 <= m <= 8 */
  ZC_GATE_PROD = 1,
  /* the polynomials of Table 1: f = g1*...*gP + gP+1 + ... + gP+A, degree P,
     tables [g1, .., gP+A], m = P + 16*A with (P, A) one of (2,0) (2,1)
     (2,2) (2,3) (3,0) (4,0) */
  ZC_GATE_SUMPROD = 2
} zc_gate;

/* Instance shape: 1 <= mu <= 30, gate in zc_gate, m used by ZC_GATE_PROD and
   ZC_GATE_SUMPROD, flags a set of ZC_FLAG_* (0 for none). */
typedef struct {
  uint32_t mu;
  uint32_t gate;
  uint32_t m;
  uint32_t flags;
} zc_shape;

/* Number of witness tables k of the gate (eq not counted), or a negative zc_status. */
int zc_table_count(const zc_shape* shape);

/* Gate degree d (the round polynomial has degree d+1, d+2 values), or a negative zc_status. */
int zc_degree(const zc_shape* shape);

/* Bytes of device workspace a proof of this shape needs (0 for an invalid shape):
   control block, the factored eq_r tables (about 4 * 2^(mu/2) elements),
   folded copies of the k witness tables (2^(mu-1) elements each), per-block
   partial sums.  256-byte alignment required. */
size_t zc_workspace_bytes(const zc_shape* shape);

/* Convert n canonical elements (canon: uint32[n][8], 16-byte aligned) into the
   internal limb-planar Montgomery form (mont_planar: uint32[8][n], pitch n),
   1 <= n <= 2^30 (the table of mu = 30; larger n returns ZC_EINVAL).
   Elements >= p are flagged (ZC_ERANGE via zc_read_error); only the control
   block of ws is used, so a workspace of any valid shape will do. */
int zc_pack(const uint32_t* canon, uint32_t* mont_planar, uint64_t n, void* ws, hipStream_t stream);

/* Inverse of zc_pack for the first n elements of a limb-planar table with the
   given pitch (canon: uint32[n][8], 16-byte aligned), 1 <= n <= 2^30,
   pitch >= n. */
int zc_unpack(const uint32_t* mont_planar, uint64_t pitch, uint32_t* canon, uint64_t n, hipStream_t stream);

/* Whole proof (Fig. 2, right).
   tables      host array of k device pointers (gate column order), each a
               packed table of 2^mu elements; READ ONLY (the folds go to ws).
   r           mu canonical elements (uint32[mu][8]); r_i >= p is flagged.
   ws          workspace of zc_workspace_bytes(shape) bytes.
   round_evals out: uint32[mu][d+2][8], G_i(0..d+1), canonical.
   challenges  out: uint32[mu][8], alpha_1..alpha_mu, canonical.
   openings    out: uint32[k+1][8], every witness table's MLE at alpha in
               column order, then eq_r(alpha), canonical. */
int zc_prove(const zc_shape* shape, const uint32_t* const* tables, const uint32_t* r, void* ws,
             uint32_t* round_evals, uint32_t* challenges, uint32_t* openings, hipStream_t stream);

/* zc_prove on tables whose limb planes are `pitch` elements apart (each
   table: uint32[8][pitch], the proof reading its first 2^mu entries), e.g. a
   2^mu-row window of a larger packed table, read in place.  pitch = 0 means
   2^mu (zc_prove); otherwise 2^mu <= pitch <= 2^30, else ZC_EINVAL.  Same
   launches and output bytes as zc_prove on a copy of the window. */
int zc_prove_pitch(const zc_shape* shape, const uint32_t* const* tables, uint64_t pitch, const uint32_t* r, void* ws,
                   uint32_t* round_evals, uint32_t* challenges, uint32_t* openings, hipStream_t stream);

/* zc_prove without a workspace argument, for callers that cannot allocate
   device memory (code under HIP graph capture, tight serving loops, hosts
   that forbid allocation).  Same launches, same output bytes as zc_prove.
   The workspace is a 32 MiB array in the library's device code, one per
   device, held from the library's first use on that device until the
   process ends; its device address is looked up once per device, on the
   first call (on the device of `stream`, the current device for the null
   stream).  No allocating call is made.
   Limit: shapes with zc_workspace_bytes(shape) <= 32 MiB (every gate up to
   mu = 17); larger shapes return ZC_ETOOBIG and enqueue nothing.
   status      out (device, may be NULL): the device-detected status of the
               proof (ZC_OK, or ZC_ERANGE for an r_i >= p), written last.
   All calls on one device share the array and its control block: calls
   that overlap in time on one device (different streams, or host threads)
   race and must be serialized by the caller.  Each call resets what must
   start cleared; the array keeps the last call's contents. */
int zc_prove_static(const zc_shape* shape, const uint32_t* const* tables, const uint32_t* r,
                    uint32_t* round_evals, uint32_t* challenges, uint32_t* openings, int32_t* status,
                    hipStream_t stream);

/* Stepping form of the same proof, same bytes as zc_prove.
   zc_round(i), 1 <= i <= mu: evaluates G_i on tables that have been folded
   i-1 times (2^(mu-i+1) live entries, pitch 2^mu), writes
   round_evals[(i-1)(d+2)..] and challenges[i-1] (same layout as zc_prove),
   and keeps alpha_i in ws.  zc_round(1) also checks r, starts the
   transcript and builds the factored eq_r tables in ws.  Must follow
   zc_fold(i-1). */
int zc_round(const zc_shape* shape, const uint32_t* const* tables, const uint32_t* r, void* ws, uint32_t i,
             uint32_t* round_evals, uint32_t* challenges, hipStream_t stream);

/* Folds the k caller tables IN PLACE (pitch 2^mu) with alpha_i:
   t[j] <- t[j] + alpha_i (t[j + h] - t[j]) for j < h = 2^(mu-i).  eq_r is
   never materialized (the library keeps it factored), so only the witness
   tables are folded.  Must follow zc_round(i).  After zc_fold(mu) entry 0 of
   each table is its opening (read it with zc_unpack, pitch 2^mu). */
int zc_fold(const zc_shape* shape, uint32_t* const* tables, void* ws, uint32_t i, hipStream_t stream);

/* ---- batches (many independent instances, one lockstep launch sequence) ----

   Each instance is a whole proof exactly as zc_prove would make it (same
   arguments, its own workspace of zc_workspace_bytes(&shape) bytes, same
   output bytes).  The instances may differ in mu and gate.  They advance
   round by round together: one round kernel per gate and step for all the
   instances of that gate, then one finisher block per instance, so that the
   per-round serial work of the instances (sum of partials, SHA-256,
   challenge) overlaps.  tile = pairs per thread in the round kernels (0
   means 4); it changes the launch shapes, not the bytes. */
typedef struct {
  zc_shape shape;
  const uint32_t* const* tables; /* host array of k device pointers, read only */
  const uint32_t* r;             /* device, mu x 8 canonical */
  void* ws;                      /* device, zc_workspace_bytes(&shape), 256-byte aligned */
  uint32_t* round_evals;         /* device outputs, as zc_prove */
  uint32_t* challenges;
  uint32_t* openings;
  uint32_t tile;
  /* elements between the limb planes of each table (0 means 2^mu, the layout
     zc_pack makes).  A larger pitch lets an instance read a 2^mu-element
     window of a larger packed table in place: tables[t] then points at the
     window's first element of plane 0 (pitch <= 2^30). */
  uint64_t pitch;
} zc_instance;

/* Bytes of device batch workspace (instance descriptors and launch
   schedule) for n instances, 1 <= n <= 65536; 0 if n is out of range. */
size_t zc_batch_workspace_bytes(uint32_t n);

/* Writes the descriptors and schedule of the n instances (host array) into
   batch_ws and synchronizes `stream`.  Checks every instance like zc_prove
   (negative zc_status, nothing written, on the first bad one). */
int zc_batch_upload(uint32_t n, const zc_instance* inst, void* batch_ws, hipStream_t stream);

/* Enqueues the batched proof of the n instances last uploaded to batch_ws
   (pass the same host array).  Only kernel launches: the sequence may be
   captured into a HIP graph and replayed while the instances' inputs stay
   where they are.  Device-detected conditions land in each instance's
   workspace (zc_read_error). */
int zc_batch_launch(uint32_t n, const zc_instance* inst, void* batch_ws, hipStream_t stream);

/* zc_batch_upload followed by zc_batch_launch. */
int zc_batch_prove(uint32_t n, const zc_instance* inst, void* batch_ws, hipStream_t stream);

/* ---- serving: instance slots advanced one round per step ----

   A pool of `slots` instance slots in device memory (zc_serve_pool_bytes).
   zc_serve_admit puts an instance into a free slot and launches its setup.
   zc_serve_step then runs one round of each listed instance, each at its
   own round, all instances of one gate sharing each launch. The step that
   runs an instance's round zc_serve_rounds(shape) also runs the rest of its
   proof; after it the outputs are complete.  The caller owns the schedule:
   instance i of a step runs rounds[i], and rounds 1..zc_serve_rounds(shape)
   of an instance must be run in order, one per step, on one stream.  A slot
   may be reused after its instance's last step (same stream, so ordered).
   Only kernel launches; no copies.  Results are the bytes zc_prove gives. */

/* Bytes of a pool of `slots` slots (1 <= slots <= 65535), 0 otherwise. */
size_t zc_serve_pool_bytes(uint32_t slots);

/* Steps (rounds run by zc_serve_step) an instance of this shape needs, or a
   negative zc_status. */
int zc_serve_rounds(const zc_shape* shape);

/* Checks the instance like zc_prove and enqueues its admission into `slot`. */
int zc_serve_admit(void* pool, uint32_t slots, uint32_t slot, const zc_instance* inst, hipStream_t stream);

/* One step for n admitted instances: slot_ids[i], rounds[i] (host arrays)
   and inst[i] (the host description the slot was admitted with). */
int zc_serve_step(void* pool, uint32_t slots, uint32_t n, const uint32_t* slot_ids, const uint32_t* rounds,
                  const zc_instance* inst, hipStream_t stream);

/* One part of one step of one admitted instance: round `round` split into
   `parts` launches (1 <= parts <= 64, 0 <= part < parts) of equal block
   counts, part `part` of them; the last part also runs the round's finisher
   (and, at round zc_serve_rounds(shape), the rest of the proof, which is
   never split: parts must be 1 there).  The parts of a round run in order
   on one stream, as whole steps do, and may interleave with other work on
   other streams: a large instance's round then takes the GPU in short
   launches.  ZC_EINVAL if the split would need more than 2048 blocks in all.
   Same bytes as zc_serve_step. */
int zc_serve_step_part(void* pool, uint32_t slots, uint32_t slot, uint32_t round, uint32_t part, uint32_t parts,
                       const zc_instance* inst, hipStream_t stream);

/* Synchronizes `stream` and returns the first device-detected error stored in
   ws (ZC_OK if none), or ZC_EHIP if the synchronization fails.  The error word
   is cleared when zc_prove or zc_round(1) starts; a workspace that has run
   neither must be zero-filled before zc_pack can report through it. */
int zc_read_error(void* ws, hipStream_t stream);

/* Static description of a status code. */
const char* zc_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* ZC_H */
