/*
 * nnvisr.h -- C-ABI of the MI355X (gfx950) frame-group enhancement library.
 *
 * The library implements the data path of NNVISR (Tong, Hu, Wang, "NNVISR: Bring
 * Neural Network Video Interpolation and Super Resolution into Video Processing
 * Framework", ACM MM 2023): Y'CbCr frames in, enhanced Y'CbCr frames out, with the
 * frame grouping the paper describes for interpolation networks, for one generic,
 * seeded extract/fusion network.
 *
 * Conventions shared by every call
 *  - Pointers named d_* and every plane pointer are HIP device memory owned by the
 *    caller (for example torch tensors).  Host pointers are marked as such.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default stream.  Work
 *    is enqueued asynchronously on it; buffers must stay valid until it completes.
 *  - Arguments are validated on the host before anything is enqueued.  On any error
 *    nothing is enqueued, no state changes, and nv_last_error() describes why.
 *  - Colour is non-linear R'G'B' and Y'CbCr of the frame format's colourspace (matrix,
 *    range and 4:2:0 chroma siting, see nv_format); by default ITU-R BT.709, limited
 *    range, left-sited chroma (co-sited with even luma columns, between luma rows 2i
 *    and 2i+1).
 *  - A context is used by one host thread at a time; calls on one context that
 *    overlap in time are not supported.  Successive calls may use different HIP
 *    streams: device work that reuses the context's workspace, or one clip stream's
 *    device state, is ordered behind the previous call that used it (the library
 *    records an event after each such call and makes the next call's stream wait on it
 *    when the stream differs), so results do not depend on the streams chosen.
 *  - No C++ exception crosses this interface.
 */
#ifndef NNVISR_H
#define NNVISR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NV_OK = 0,
  NV_E_INVALID = 1,      /* bad argument: null pointer, size, format, pitch, state */
  NV_E_UNSUPPORTED = 2,  /* valid but not implemented (e.g. a precision, a format) */
  NV_E_NOMEM = 3,        /* device allocation failed */
  NV_E_DEVICE = 4,       /* a HIP call failed; see nv_last_error() */
  NV_E_BUSY = 5          /* serving queue full / admission refused */
} nv_status;

/* Arithmetic of the network's convolutions (the offset head is float-class, see
 * NV_FLAG_HEAD_FP32; the bilinear sampling weights and all pixel-format stages are FP32
 * in every mode).  FP16 / BF16 store the
 * feature maps in that type and run every other conv on it with FP32 accumulation.
 * NV_FP8_E4M3 (64 channels only) stores feature maps in FP16, runs the residual-block
 * convs (and with NV_FLAG_FP8_FUSION the deformable conv and the pixel-shuffle conv)
 * with OCP e4m3 operands (per output channel weight scales max|W|/448, one static
 * activation scale per layer, see nv_calibrate) and FP32 accumulation, and every other
 * conv as in FP16. */
typedef enum { NV_FP32 = 0, NV_FP16 = 1, NV_BF16 = 2, NV_FP8_E4M3 = 3 } nv_precision;

/* Network flags of the paper's network-integration section (section 3.1):
 * Interpolation doubles the frame rate, Extra frame means the network takes n+1
 * frames, Double frame means it emits 2n frames (without it, and with Interpolation,
 * the input frames are output unchanged and the network's outputs are the frames
 * between them).  Supported: Interpolation|Extra frame|Double frame (groups [a, b], two
 * outputs per input frame), Interpolation|Extra frame (scale 1 only: input frame a passes
 * through, then the frame between a and b), and none (each frame enhanced alone, one
 * output per input frame). */
enum { NV_FLAG_INTERP = 1, NV_FLAG_EXTRA = 2, NV_FLAG_DOUBLE = 4 };

/* Offset head arithmetic (a library option, not one of the paper's flags).  The head
 * (both convs of the offset/mask prediction) is float-class in every precision.  In
 * FP32 mode it runs on float MFMA.  In the FP16 / BF16 / FP8 modes it runs by default on
 * float16 MFMA with each weight carried as two float16 parts (hi + lo, about 22 bits)
 * and the float input of its second conv staged the same way, products exact and
 * accumulated in float; NV_FLAG_HEAD_FP32 in nv_net_config.flags selects float MFMA
 * there too. */
enum { NV_FLAG_HEAD_FP32 = 8 };

/* FP8 scope (library option, NV_FP8_E4M3 only).  By default FP8 covers the residual
 * blocks of the extract stage (the bulk of the work); the deformable conv and the
 * pixel-shuffle conv run as in FP16 mode, which keeps every output frame of the
 * 1920x1080, C = 64, R = 10 network above 50 dB PSNR against the FP64 reference.
 * NV_FLAG_FP8_FUSION puts those two convs on e4m3 too (faster, measured 45.8 dB on that
 * network's worst window). */
enum { NV_FLAG_FP8_FUSION = 16 };

/* Colourspace of a frame (section 3.1, colourspace paragraph: the same code values mean
 * different colours under different colourspaces, so the matrix and range travel with
 * the frame and a network is trained for one colourspace).
 *  matrix      NV_MATRIX_BT709 (ITU-R BT.709), NV_MATRIX_BT601 (BT.601), NV_MATRIX_BT2020
 *              (BT.2020 non-constant luminance): the luma weights Kr, Kb of
 *              Y' = Kr R' + (1 - Kr - Kb) G' + Kb B', Cb' = (B' - Y') / (2 (1 - Kb)),
 *              Cr' = (R' - Y') / (2 (1 - Kr)).
 *  range       NV_RANGE_LIMITED: Y = (219 Y' + 16) 2^(b-8), C = (224 C' + 128) 2^(b-8);
 *              NV_RANGE_FULL: Y = (2^b - 1) Y', C = (2^b - 1) C' + 2^(b-1).
 *  chroma_loc  4:2:0 only.  NV_SITING_LEFT (MPEG-2): chroma sample (i, j) at luma column
 *              2j, halfway between rows 2i and 2i+1; bilinear upsampling, (1/4, 1/2, 1/4) x
 *              (1/2, 1/2) downsampling.  NV_SITING_CENTER (MPEG-1 / JPEG): at the centre of
 *              its 2x2 luma block; bilinear upsampling, 2x2 box downsampling.
 * Zero in all three is BT.709, limited range, left siting. */
enum { NV_MATRIX_BT709 = 0, NV_MATRIX_BT601 = 1, NV_MATRIX_BT2020 = 2 };
enum { NV_RANGE_LIMITED = 0, NV_RANGE_FULL = 1 };
enum { NV_SITING_LEFT = 0, NV_SITING_CENTER = 1 };

/* Frame format.  width/height are luma sizes (even for 4:2:0); bits is 8 (uint8
 * samples) or 10 (uint16 little-endian samples holding the code in the low 10 bits;
 * the upper 6 bits are ignored on input and written as zero); chroma is 420 or 444;
 * matrix, range and chroma_loc as above. */
typedef struct {
  int32_t width, height, bits, chroma;
  int32_t matrix, range, chroma_loc;
} nv_format;

/* Planar Y, Cb, Cr.  pitch_bytes[i] is the distance between rows of plane i. */
typedef struct {
  void* data[3];
  int64_t pitch_bytes[3];
} nv_planes;

/* Network shape and task.  channels C (32 or 64; 64 for NV_FP8_E4M3), res_blocks R
 * (0..64), offset_groups G (even, 2C divisible by G, 2C/G a multiple of 4), align must
 * be 8.  The task (section 3.2, end-user usage) is set by the scale factors and the
 * flags: scale is the horizontal factor and scale_v the vertical one (1 or 2 each;
 * scale_v 0 = scale), flags as above, optionally with NV_FLAG_HEAD_FP32 and (FP8 only)
 * NV_FLAG_FP8_FUSION.  The tasks of that section: scale 1 with no flags denoises; scale
 * 2 with no flags is super-resolution; scale 1, scale_v 2 with no flags deinterlaces;
 * scale 1 with Interpolation|Extra frame interpolates with the input frames passed
 * through; scale 1 with all three interpolates and denoises; scale 2 with all three is
 * space-time super-resolution (the only task for NV_FP8_E4M3, nv_enhance_batch and the
 * batched paths).  Output frames are the input format at scale x width, scale_v x height.
 * The weight blob omits off1, off2 and dcn for networks without Interpolation, and its
 * up conv has scale x scale_v x C outputs (a plain conv when both are 1).  matrix and range name the
 * colourspace the weights were trained for (section 3.1: networks are trained per
 * colourspace and the one matching the clip is used): the enhancement calls of the
 * context (group, clip stream, batch, calibration) refuse frames of another matrix or
 * range with NV_E_UNSUPPORTED, so a caller holding one context per colourspace selects
 * the network by the clip's format.  The pixel-format stages alone (nv_unpack, nv_pack,
 * nv_scene_metric) take any colourspace.  levels > 1 (interpolating networks in FP32,
 * FP16 or BF16; not in nv_enhance_batch) makes the extract stage output a feature
 * pyramid (section 3.1): level l >= 2 is conv + LReLU of the 2x2 mean pool of level
 * l-1, and the alignment runs from the coarsest level down, each level adding twice
 * the x2 resize of the coarser level's offsets to its own and the x2 resize of the
 * coarser aligned features to its own; the blob then holds "down" (C x C) for levels
 * 2..L after the residual blocks, and off1, off2, dcn for levels 2..L after level 1's. */
typedef struct {
  int32_t channels, res_blocks, offset_groups, scale, align;
  uint32_t flags;
  int32_t precision;     /* nv_precision */
  int32_t matrix, range; /* colourspace of the training data: NV_MATRIX_*, NV_RANGE_* */
  int32_t scale_v;       /* vertical scale factor, 0 = the same as scale */
  int32_t levels;        /* feature-pyramid levels, 0 or 1 = one, at most 4 */
} nv_net_config;

/* Scene-change rule: frame t starts a scene when
 *   SAD_t > mad_thresh_8bit * 2^(bits-8) * N   and   HD_t * hist_frac_den > 2 * N * hist_frac_num
 * where N = width*height, SAD_t = sum |Y_t - Y_{t-1}| over luma codes and HD_t the L1
 * distance of the 64-bin luma histograms (bin = code >> (bits-6)).  enable = 0 leaves
 * the decision to the external per-frame flags alone. */
typedef struct {
  int32_t mad_thresh_8bit, hist_frac_num, hist_frac_den, enable;
} nv_scene_params;

typedef struct nv_context nv_context;
typedef struct nv_stream nv_stream;

/* ---------------------------------------------------------------- context ---- */

/* Create a context on HIP device `device` for one network (section 3.1, network
 * integration: the network is supplied once and split into an extract stage run per
 * frame and a fusion stage run per frame group).  `weights` (HOST memory, float32,
 * n_floats long) is the flat weight blob in this tensor order, each conv 3x3 OIHW
 * followed by its bias: conv_in (C,3), R x [block.a (C,C), block.b (C,C)],
 * off1 (C,2C), off2 (27G,C), dcn (C,2C), up (4C,C), hr (3,C) for the default task (see
 * nv_net_config for the others).  The library copies and repacks it; the caller may free
 * it on return. */
nv_status nv_context_create(int32_t device, const nv_net_config* cfg, const float* weights,
                            size_t n_floats, nv_context** out);
nv_status nv_context_destroy(nv_context* ctx);

/* Thread-local, NUL-terminated description of the last error on this thread. */
const char* nv_last_error(void);

/* Number of floats the weight blob of `cfg` must hold (0 if cfg is invalid). */
size_t nv_weight_count(const nv_net_config* cfg);

/* FP8 activation scales.  An NV_FP8_E4M3 context quantises the input of each of its
 * FP8 layers (in this order: block.a and block.b of each residual block, then with
 * NV_FLAG_FP8_FUSION the deformable conv and the pixel-shuffle conv; 2R or 2R + 2
 * layers) with a static scale amax / 448, where amax
 * is the largest |input| the layer saw during calibration; the scales stay fixed
 * afterwards, so a frame's result does not depend on what it is batched with.  Every
 * enhancement call of an FP8 context fails with NV_E_INVALID until one of these has
 * been called.
 *
 * nv_calibrate runs the network over the n_frames (>= 2, device planes of format fmt)
 * as consecutive frame groups (0,1), (1,2), ... without scene detection, and sets each
 * layer's amax to the largest |input| seen (the layers after it already use the
 * updated scales).  It uses the context's workspace, enqueues on `stream` and does not
 * synchronise.  NV_E_INVALID for contexts of other precisions.
 *
 * nv_fp8_scales reads (set = 0) or writes (set = 1) the n (2R or 2R + 2) amax values in
 * host memory, e.g. to reuse one calibration in other contexts; it synchronises
 * `stream`.  Written values must be finite and >= 0 (0 means scale 1). */
nv_status nv_calibrate(nv_context* ctx, const nv_format* fmt, const nv_planes* frames, int32_t n_frames,
                       void* stream);
nv_status nv_fp8_scales(nv_context* ctx, float* amax, int32_t n, int32_t set, void* stream);

/* ------------------------------------------------- pixel-format stages ---- */

/* Unpack one frame (section 3.1, pixel formats): decode codes, upsample 4:2:0 chroma
 * bilinearly for its siting, normalise by its range and apply its matrix's inverse (no
 * clamp), and write planar float32
 * R'G'B' d_rgb[3][hp][wp] (plane stride hp*wp floats).  hp >= height and wp >= width, wp a
 * multiple of 4, d_rgb 16-byte aligned;
 * rows/columns beyond the frame replicate the last row/column (alignment padding). */
nv_status nv_unpack(const nv_format* fmt, const nv_planes* in, float* d_rgb, int32_t hp,
                    int32_t wp, void* stream);

/* Requantise planar float32 R'G'B' to a frame of format `fmt` (section 3.1, pixel
 * formats: the enhanced frames leave in the clip's Y'CbCr format): clamp R'G'B' to [0,1],
 * the format's forward matrix and range, 4:2:0 chroma by its siting's downsampling
 * filter with replicated edges, code = clamp(floor(v + 1/2), 0, 2^bits - 1).  d_rgb
 * is [3][rh][rw] (rh >= fmt->height, rw >= fmt->width, rw a multiple of 4, d_rgb
 * 16-byte aligned); only the top-left fmt->height x fmt->width region is read (crop). */
nv_status nv_pack(const nv_format* fmt, const float* d_rgb, int32_t rh, int32_t rw,
                  const nv_planes* out, void* stream);

/* Integer scene metric of frame `cur` against `prev` (sections 3.2 and 3.3: groups
 * stay inside a scene).  Writes device values: *d_sad (uint64), d_hist[64] (uint32,
 * histogram of cur), *d_hd (uint32), *d_cut (uint32, 0/1).  prev == NULL (first frame)
 * or d_hist_prev == NULL yields sad = hd = 0 and cut = 1.  external_cut: -1 none,
 * 0 or 1 OR-ed into the decision. */
nv_status nv_scene_metric(const nv_format* fmt, const nv_planes* prev, const nv_planes* cur,
                          const uint32_t* d_hist_prev, const nv_scene_params* params,
                          int32_t external_cut, uint64_t* d_sad, uint32_t* d_hist,
                          uint32_t* d_hd, uint32_t* d_cut, void* stream);

/* --------------------------------------------------------- network ---- */

/* Bytes per feature element: 4 (float32) for NV_FP32 contexts, 2 (float16 or bfloat16,
 * matching the precision) otherwise.  Features are NHWC [hp][wp][C]. */
int32_t nv_feature_elem_bytes(const nv_context* ctx);

/* Bytes of one frame's features at padded size hp x wp: every level of the context's
 * feature pyramid, level 1 ([hp][wp][C]) first, then level l = 2..levels as
 * [hp >> (l-1)][wp >> (l-1)][C], back to back.  0 on a NULL context. */
size_t nv_feature_bytes(const nv_context* ctx, int32_t hp, int32_t wp);

/* Extract stage (section 3.1: per frame, the feature pyramid) from planar float32
 * R'G'B' d_rgb[3][hp][wp] (hp, wp multiples of 8) into the context's feature type at
 * d_feat (nv_feature_bytes(ctx, hp, wp) bytes; level 1 is NHWC [hp][wp][C]). */
nv_status nv_extract(nv_context* ctx, const float* d_rgb, int32_t hp, int32_t wp,
                     void* d_feat, void* stream);

/* Fusion stage of the frame group [a, b] (section 3.1).  Produces float32 HR R'G'B'
 * planes [3][2hp][2wp] for each set bit of out_mask: bit 0 -> t = 0 (d_hr[0]),
 * bit 1 -> t = 1/2 (d_hr[1]), bit 2 -> t = 1 (d_hr[2]).  If d_sel is not NULL and
 * *d_sel != 0 (device uint32, e.g. a scene-cut flag) the group is [a, a]: frame b's
 * features and pixels are replaced by frame a's (section 3.3: the last frame of a
 * scene is duplicated).  Optional device outputs for inspection (NULL to skip):
 * d_offsets [hp][wp][ldo] with ldo = 16*ceil(27G/16): channel 2(9g+k) dy, 2(9g+k)+1
 * dx, 18G + 9g + k the sigmoid mask (float32); d_fmid [hp][wp][C] the aligned features
 * (feature type). */
nv_status nv_fuse(nv_context* ctx, const float* d_rgb_a, const float* d_rgb_b,
                  const void* d_feat_a, const void* d_feat_b, int32_t hp, int32_t wp,
                  const uint32_t* d_sel, uint32_t out_mask, float* const d_hr[3],
                  float* d_offsets, void* d_fmid, void* stream);

/* --------------------------------------------------------- end to end ---- */

/* One frame group (section 3.1: a frame group in, enhanced frames out): two frames in,
 * three frames out (t = 0, 1/2, 1) of the output format (the input format scaled by the
 * task's factors; twice the width and height for the space-time task of section 3.2).
 * Without Double frame the t = 0 and t = 1 outputs are the inputs passed through.
 * NV_E_UNSUPPORTED for networks without Interpolation (no groups: use a clip stream).
 * in[2] and out[3] are HOST arrays of device planes. */
nv_status nv_enhance_group(nv_context* ctx, const nv_format* fmt, const nv_planes in[2],
                           const nv_planes out[3], void* stream);

/* Allocation-free form of nv_enhance_group, for callers that cannot allocate device
 * memory during the call (work recorded under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, validation and results (bit for bit)
 * as nv_enhance_group, but the call allocates nothing: every temporary (R'G'B' of both
 * inputs, their features, the offset head's hidden map, offsets and mask, aligned and
 * high-resolution features, HR R'G'B') lives in a fixed device buffer of
 * NV_STATIC_SCRATCH_BYTES per device, a static of the library that the HIP runtime
 * allocates with the library's code object on each device that loads it and that stays
 * allocated until the process ends; its address is looked up when a context is created
 * on the device.  A group whose temporaries exceed the buffer (C = 64 in FP32 needs
 * about 3.3 KB per padded pixel, so about 20 000 padded pixels, e.g. 160x128) returns
 * NV_E_INVALID without enqueuing anything.  Every call on one device uses the same
 * buffer, from every context on that device: calls that overlap in time on one device
 * (on different HIP streams, from different contexts or threads) race and corrupt each
 * other's results.  Calls are not timed by nv_profile_enable. */
#define NV_STATIC_SCRATCH_BYTES (64u << 20)
nv_status nv_enhance_group_static(nv_context* ctx, const nv_format* fmt, const nv_planes in[2],
                                  const nv_planes out[3], void* stream);

/* Clip-level streaming (section 3.2: one function from clip to enhanced clip).
 * push(t) unpacks frame t, runs the scene metric and the extract stage, and emits the
 * two outputs of group t-1 (frame t-1 at t = 0, enhanced or passed through without
 * Double frame, then the interpolated frame), so *n_out is 0 for t = 0 and 2
 * afterwards; end() emits the last group's two outputs.  For a network without
 * Interpolation push(t) emits frame t enhanced (*n_out = 1, out needs one entry) and
 * end() emits nothing.
 * The cut decision stays on the device: no host synchronisation per frame. */
nv_status nv_stream_open(nv_context* ctx, const nv_format* fmt, const nv_scene_params* params,
                         nv_stream** out);
nv_status nv_stream_push(nv_stream* s, const nv_planes* frame, int32_t external_cut,
                         const nv_planes out[2], int32_t* n_out, void* stream);
nv_status nv_stream_end(nv_stream* s, const nv_planes out[2], int32_t* n_out, void* stream);
nv_status nv_stream_close(nv_stream* s);

/* Restart a stream at frame 0 (a new clip of the same format) keeping its device
 * buffers; the next push starts a new scene. */
nv_status nv_stream_reset(nv_stream* s);

/* Copy the device cut flags of the frames pushed so far into host memory
 * (cuts[0..n-1], n <= frames pushed); synchronises `stream`. */
nv_status nv_stream_cuts(nv_stream* s, uint32_t* host_cuts, int32_t n, void* stream);

/* ------------------------------------------- general n, batches of b groups ---- */

/* A clip grouped for a network that consumes n frames per run, with the Extra frame
 * (n + 1 inputs) and Double frame (2n outputs) flags of section 3.1, run in batches of b
 * groups over the frame store of section 3.3 (Fig. 1).  The network's fusion is pairwise,
 * so a group's outputs are, for each frame it consumes, the frame itself (t = 0) and the
 * frame between it and the group's next input (t = 1/2); over a clip every input frame
 * gives these two outputs once, in input order, exactly as with nv_stream_push.
 *
 * Grouping (section 3.3): groups never cross a scene cut; the input after a scene's last
 * frame is that frame again; a last group short of frames recycles the previous group's
 * last frames; a scene shorter than n frames repeats its last frame.  A frame's outputs
 * come from the first group that consumes it.
 *
 * Frame store (Fig. 1): n b + b positions of R'G'B' and features.  For the block of b
 * groups starting at frame f0, frame f0 + i n (i = 0..b) sits at position b - 1 + i and
 * frame f0 + i n + k (k = 1..n-1) at 2b + (k - 1) b + i, so each network input of the b
 * groups is b consecutive positions and no frame is stored twice; after a full block the
 * last frame is copied into the chain start (position b - 1, the figure's "6 to 5") and
 * the next block starts from it.
 *
 * push() runs the scene metric, reads the frame's cut flag back to the host (the grouping
 * depends on where scenes end, so push synchronises `stream`), then finishes the previous
 * scene's groups if the frame starts a new scene, and stores and extracts the frame; when
 * a block of b groups is complete its groups run.  end() runs the last scene's remaining
 * groups.  out (HOST array of out_cap device planes of the output format) receives the
 * emitted frames in order, *n_out of them; 2 n b entries always suffice.  n >= 1, b >= 1,
 * n b + b <= 64.  The clip keeps its frame store on the device until nv_clip_close.
 *
 * nv_clip_trace copies what the clip ran, for inspection: per batch, the kind (0 a full
 * block, 1 the remaining groups of a scene), the number of groups g, g x (n + 1) input
 * frame numbers, and the frame number held at each of the n b + b store positions when
 * the batch ran (-1 empty).  *len receives the total length; at most cap values are
 * written to buf (HOST). */
typedef struct nv_clip nv_clip;
nv_status nv_clip_open(nv_context* ctx, const nv_format* fmt, const nv_scene_params* params, int32_t n,
                       int32_t b, nv_clip** out);
nv_status nv_clip_push(nv_clip* clip, const nv_planes* frame, int32_t external_cut, const nv_planes* out,
                       int32_t out_cap, int32_t* n_out, void* stream);
nv_status nv_clip_end(nv_clip* clip, const nv_planes* out, int32_t out_cap, int32_t* n_out, void* stream);
nv_status nv_clip_trace(const nv_clip* clip, int32_t* buf, int32_t cap, int32_t* len);
nv_status nv_clip_close(nv_clip* clip);

/* Device bytes a stream of this format keeps resident (for admission control): the
 * frame store of section 3.3 for n = 1 (the overlap frame's pixels and features, two
 * ring slots) plus the scene state (previous luma plane, histogram, cut flags).  The
 * context workspace and the batch workspace (nv_batch_footprint) are not included. */
nv_status nv_stream_footprint(const nv_context* ctx, const nv_format* fmt, size_t* bytes);

/* ------------------------------------------------------------ batching ---- */

enum { NV_BATCH_MAX_FRAMES = 256, NV_BATCH_MAX_GROUPS = 512, NV_BATCH_MAX_CHAIN = 16 };

/* One request of a batch: n_frames (1..NV_BATCH_MAX_CHAIN) consecutive frames of one
 * clip stream, processed exactly as n_frames calls of nv_stream_push (external_cut[j],
 * or -1 for every frame when external_cut is NULL), followed by nv_stream_end when
 * end_of_clip != 0.  The frames of a request share the paper's batched frame store for
 * n = 1 (section 3.3, Fig. 1): b groups read b + 1 stored frames, none duplicated.
 * out[] holds room for 2 * n_frames + 2 output frames (in emission order); *n_out
 * receives the number written.  frames, external_cut, out and n_out are HOST arrays;
 * the planes they describe are device memory. */
typedef struct {
  nv_stream* stream;
  int32_t n_frames;
  const nv_planes* frames;
  const int32_t* external_cut;
  const nv_planes* out;
  int32_t* n_out;
  int32_t end_of_clip;
} nv_batch_req;

/* Run many streams' requests (any formats and sizes) together: every stage is one
 * persistent launch over all images of the batch, and the launch sequence is recorded
 * once into a HIP graph and replayed for later batches (the per-batch job tables are
 * uploaded before each replay).  Results are bit-identical to per-stream calls.  The
 * streams of one call must be distinct and belong to ctx; at most NV_BATCH_MAX_FRAMES
 * frames and NV_BATCH_MAX_GROUPS groups per call.  Device workspace grows to the largest
 * batch seen (see nv_batch_footprint). */
nv_status nv_enhance_batch(nv_context* ctx, const nv_batch_req* reqs, int32_t n, void* stream);

/* on != 0 (the default): record and replay the batch graph; 0: launch directly. */
nv_status nv_batch_graph(nv_context* ctx, int32_t on);

/* Device bytes the batch pools take per padded LR pixel (section 3.3: a batch holds its
 * groups' temporaries and its frames' features): *per_group for each group of the batch
 * (offset-head hidden map, offsets, aligned features, HR features, HR R'G'B') and
 * *per_frame for each frame, before each buffer is rounded up to 256 bytes.  A server
 * adds them to nv_stream_footprint when it admits streams to batched calls. */
nv_status nv_batch_bytes_per_px(const nv_context* ctx, size_t* per_group, size_t* per_frame);

/* Device bytes of batch workspace currently held by ctx. */
nv_status nv_batch_footprint(const nv_context* ctx, size_t* bytes);

/* Autotuner: times each candidate workgroup tile (rows per wave, waves along the output
 * channels) of the residual-block conv, the pixel-shuffle conv, the offset head and the
 * DCN on an hp x wp frame and keeps the fastest in ctx.  The DCN candidates include its
 * forms that read the sampling corners from an LDS copy of their window (all forms give
 * bit-identical results); before any tuning a context uses default tiles, for the DCN
 * the staged form wherever it applies.  When the environment variable
 * NNVISR_TUNE_CACHE names a file, results are looked up there first (key: precision,
 * channels, hp, wp) and appended after timing.  A human-readable summary is written to
 * report (HOST, may be NULL). */
nv_status nv_autotune(nv_context* ctx, int32_t hp, int32_t wp, void* stream, char* report,
                      size_t report_len);

/* ------------------------------------------------------- kernel timing ---- */

/* Kinds of launches the library times when profiling is on. */
enum {
  NV_K_UNPACK = 0, NV_K_SCENE = 1, NV_K_CONV_IN = 2, NV_K_CONV_BLOCK = 3, NV_K_OFF1 = 4,
  NV_K_OFF2 = 5, NV_K_DCN = 6, NV_K_UP = 7, NV_K_HR = 8, NV_K_PACK = 9,
  NV_K_RESBLOCK = 10,   /* both convs of a residual block in one launch (16-bit maps, C = 64) */
  NV_K_POOL = 11,       /* 2x2 mean pool starting a feature-pyramid level */
  NV_K_CASCADE = 12,    /* x2 resize of a coarser pyramid level's offsets or aligned features */
  NV_K_COUNT = 13
};

/* on != 0: from now on every launch the context makes (including those of its streams)
 * is bracketed by HIP events recorded on the launch's stream; on == 0 stops recording.
 * Enabling clears previous records.  Batched calls are timed when their graph replay
 * is off (nv_batch_graph); a replayed graph is not. */
nv_status nv_profile_enable(nv_context* ctx, int32_t on);

/* Totals per kind since the last enable: launches[k] and device milliseconds ms[k]
 * (HOST arrays of NV_K_COUNT entries).  Waits for the recorded events to complete. */
nv_status nv_profile_read(nv_context* ctx, int64_t* launches, double* ms);

/* Short name of a kind ("conv_block", ...), or "" when out of range. */
const char* nv_profile_kind_name(int32_t kind);

#ifdef __cplusplus
}
#endif
#endif /* NNVISR_H */
